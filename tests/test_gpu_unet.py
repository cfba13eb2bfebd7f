"""The HIP U-Net (BF16 weights/activations, FP32 accumulation) against the
FP64 oracle: forward output, loss, parameter gradient, Adam update, and a
short training run.  Two architectures: 3 levels on a 17 x 17 grid, and the
continuation benchmark's 4 levels / 32 base channels (32-256 channels, the
384-channel decoder input) on 65 x 65, whose 256- and 384-channel layers
take the weight gradient's capped pixel split; one forward pass and one
gradient at the benchmark's 513 x 513.  Tolerances follow BF16 storage (8 significant bits):
outputs and gradients within a few per cent in the L2 norm."""
import numpy as np
import pytest

import oracle
from oracle import continuation as oc
from oracle import unet as U
from paper_1204_5125_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LEVELS, BASE, N, SIDE = 3, 32, 17, 4.0
# (levels, base channels, grid nodes per axis, side)
ARCHS = [(3, 32, 17, 4.0), (4, 32, 65, 8.0)]
ARCH_IDS = ["3lev-17", "4lev-65"]


@pytest.fixture(scope="module")
def glnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5125_amd import glnk as g
    g.lib()
    return g


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pair(seed, mu=0.6, N=N, SIDE=SIDE):
    """(mesh, psi, base start, aligned target)."""
    mo = oracle.Mesh(2, (N, N), (SIDE, SIDE), mu=mu)
    psi = inputs.random_phase_state(mo.n, seed=seed)
    psb = psi * (1.0 + 0.02 * inputs.random_complex(mo.n, seed=seed + 200))
    tgt = psi * (1.0 + 0.03 * inputs.random_complex(mo.n, seed=seed + 100)) * np.exp(0.4j)
    tgt = oc.secant_predict(mo, psi, tgt, -1.0)  # aligned to psi
    return mo, psi, psb, tgt


def params(glnk, seed=7, LEVELS=LEVELS, BASE=BASE):
    shapes = glnk.unet_layer_shapes(LEVELS, BASE)
    assert shapes == U.layer_specs(LEVELS, BASE)
    return inputs.unet_init(shapes, seed=seed, head_scale=1.0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("arch", ARCHS, ids=ARCH_IDS)
def test_forward_matches_oracle(glnk, arch):
    LEVELS, BASE, N, SIDE = arch
    mo, psi, psb, _ = pair(1, N=N, SIDE=SIDE)
    theta = params(glnk, LEVELS=LEVELS, BASE=BASE)
    net = glnk.UNet(LEVELS, BASE)
    assert net.n_params == U.num_params(U.layer_specs(LEVELS, BASE))
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    mg = glnk.Mesh(2, (N, N), (SIDE, SIDE), mu=0.6)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    net.predict(mg, dev(psi), dev(psb), 0.6, 0.02, out)
    og = (host(out) - psb) / 0.02
    oo = U.predict(theta.astype(np.float64), U.layer_specs(LEVELS, BASE), LEVELS, psi, psb, 0.6, 0.02, N)
    oo = (oo - psb) / 0.02
    e = rel(og, oo)
    assert e < 3e-2, e


def test_forward_full_size(glnk):
    """One forward pass of the benchmark's network (4 levels, 32 base
    channels) on the 513 x 513 grid against the FP64 oracle."""
    LEVELS, BASE, N, SIDE = 4, 32, 513, 8.0
    mo, psi, psb, _ = pair(4, N=N, SIDE=SIDE)
    theta = params(glnk, seed=12, LEVELS=LEVELS, BASE=BASE)
    net = glnk.UNet(LEVELS, BASE)
    net.set_params(theta)
    mg = glnk.Mesh(2, (N, N), (SIDE, SIDE), mu=0.6)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    net.predict(mg, dev(psi), dev(psb), 0.6, 0.02, out)
    og = (host(out) - psb) / 0.02
    oo = U.predict(theta.astype(np.float64), U.layer_specs(LEVELS, BASE), LEVELS, psi, psb, 0.6, 0.02, N)
    e = rel(og, (oo - psb) / 0.02)
    assert e < 3e-2, e


# the gradient also at the benchmark's 513 x 513, where the first level's
# convolutions run with 128-pixel work-groups and the deeper ones split their
# reduction over a work-group's waves (at 17 and 65 every layer splits)
@pytest.mark.parametrize("arch", ARCHS + [(4, 32, 513, 8.0)], ids=ARCH_IDS + ["4lev-513"])
def test_loss_and_gradient_match_oracle(glnk, arch):
    LEVELS, BASE, N, SIDE = arch
    mo, psi, psb, tgt = pair(2, N=N, SIDE=SIDE)
    theta = params(glnk, seed=8, LEVELS=LEVELS, BASE=BASE)
    specs = U.layer_specs(LEVELS, BASE)
    net = glnk.UNet(LEVELS, BASE)
    net.set_params(theta)
    mg = glnk.Mesh(2, (N, N), (SIDE, SIDE), mu=0.6)
    Lg, gg = net.loss_grad(mg, dev(psi), dev(psb), 0.6, 0.02, dev(tgt))
    Lo, go = U.loss_and_grad(theta.astype(np.float64), specs, LEVELS, psi, psb, 0.6, 0.02, tgt,
                             U.volumes(N, SIDE), N)
    assert Lg == pytest.approx(Lo, rel=3e-2)
    cos = gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go))
    eg = rel(gg, go)
    assert cos > 0.995 and eg < 0.1, (cos, eg)
    # layer by layer (weights and bias of each convolution)
    o = 0
    for ci, co, k in specs:
        nw = co * k * k * ci
        el = rel(gg[o:o + nw], go[o:o + nw])
        assert el < 0.15, ((ci, co, k), el)
        o += nw + co


@pytest.mark.parametrize("arch", ARCHS, ids=ARCH_IDS)
def test_adam_step_matches_oracle_update(glnk, arch):
    LEVELS, BASE, N, SIDE = arch
    mo, psi, psb, tgt = pair(3, N=N, SIDE=SIDE)
    theta = params(glnk, seed=9, LEVELS=LEVELS, BASE=BASE)
    net = glnk.UNet(LEVELS, BASE)
    net.set_params(theta)
    mg = glnk.Mesh(2, (N, N), (SIDE, SIDE), mu=0.6)
    _, g = net.loss_grad(mg, dev(psi), dev(psb), 0.6, 0.02, dev(tgt))
    net.train_step(mg, [dev(psi)], [dev(psb)], [0.6], [0.02], [dev(tgt)], lr=1e-3)
    th1 = net.get_params()
    m, v = np.zeros(theta.size), np.zeros(theta.size)
    want = U.adam_step(theta.astype(np.float64), m, v, g.astype(np.float64), 1, lr=1e-3)
    assert np.abs(th1 - want).max() < 1e-3 * 1e-3


def test_training_reduces_the_loss(glnk):
    """A learnable target (the correction (0.5 - 0.3i) psi of a constant
    start): 60 Adam steps on four samples halve the loss."""
    def learnable(seed, mu):
        mo = oracle.Mesh(2, (N, N), (SIDE, SIDE), mu=mu)
        psi = inputs.random_phase_state(mo.n, seed=seed)
        return mo, psi, psi, psi + 0.02 * (0.5 - 0.3j) * psi

    pairs = [learnable(10 + k, 0.5 + 0.1 * k) for k in range(4)]
    net = glnk.UNet(LEVELS, BASE)
    net.set_params(params(glnk, seed=11) * 0.5)
    mg = glnk.Mesh(2, (N, N), (SIDE, SIDE), mu=0.6)
    ps = [dev(p) for _, p, _, _ in pairs]
    bs = [dev(b) for _, _, b, _ in pairs]
    ts = [dev(t) for _, _, _, t in pairs]
    mus = [0.5 + 0.1 * k for k in range(4)]
    first = net.train_step(mg, ps, bs, mus, [0.02] * 4, ts, lr=2e-3)
    for _ in range(60):
        last = net.train_step(mg, ps, bs, mus, [0.02] * 4, ts, lr=2e-3)
    assert last < 0.5 * first
