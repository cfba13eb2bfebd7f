"""Learned Newton start for the mu-continuation (an extension beyond the paper
of the continuation in Sec. 4): the library's U-Net corrects the secant start.
Training data come from a seeded continuation sweep; training runs the
library's own kernels; at run time the corrected start is used unless the
plain secant start has the smaller GL residual.

Host orchestration only: predictions, residuals, alignment and training all
run in libglnk kernels.
"""
import numpy as np

from . import continuation, glnk, inputs


def sweep(mesh, mus, psi0, **kw):
    """Converged states (mu, tensor) along the field values mus.  Where the
    continuation fails (Newton does not converge even after step halvings,
    e.g. where the branch ends), it restarts from the last converged state at
    the next field value of the list."""
    records, states = [], []
    start, todo, seg = psi0, list(mus), 0
    while todo:
        recs, _, st = continuation.continuation_path(mesh, start, todo, keep=True, **kw)
        records += recs
        steps = {r["mu"]: r["newton_steps"] for r in recs if r["status"] == 0}
        states += [(mu, psi, seg, steps.get(mu, 0)) for mu, psi in st]
        if recs[-1]["status"] == 0:
            break
        todo = [m for m in todo if m > recs[-1]["mu"] + 1e-12]
        if states:
            start = states[-1][1]
        seg += 1
    return records, states


def secant_base(mesh, psi, prev, mu_prev, mu, mu_next, out):
    """The continuation's secant start at mu_next (psi itself without history)."""
    if prev is None:
        out.copy_(psi)
    else:
        glnk.gl_secant_predict(mesh, psi, prev, (mu_next - mu) / (mu - mu_prev), out)
    return out


def make_pairs(mesh, states, strides=(1, 2, 3), jump_newton=6):
    """Training samples (psi_i, secant start, aligned psi_j, mu_i, mu_j - mu_i)
    for j = i + s inside one continuation segment, leaving out spans where the
    branch jumped (a state in (i, j] needed more than jump_newton Newton
    steps) and targets that needed no Newton step (the start was already the
    solution, e.g. the normal state psi = 0: nothing to learn).  The target is rotated by the global phase that aligns it with
    psi_i (gl_secant_predict with ratio -1 gives e^{i chi} target); the secant
    start uses psi_{i-1}."""
    import torch
    samples = []
    for s in strides:
        for i in range(len(states) - s):
            mu_i, psi_i, seg, _ = states[i]
            mu_j, psi_j, seg_j, _ = states[i + s]
            if seg_j != seg or any(states[k][3] > jump_newton for k in range(i, i + s + 1)):
                continue
            if states[i + s][3] == 0:
                continue
            t = torch.empty_like(psi_i)
            glnk.gl_secant_predict(mesh, psi_i, psi_j, -1.0, t)
            b = torch.empty_like(psi_i)
            if i > 0 and states[i - 1][2] == seg and states[i][3] <= jump_newton:
                secant_base(mesh, psi_i, states[i - 1][1], states[i - 1][0], mu_i, mu_j, b)
            else:
                b.copy_(psi_i)
            samples.append((psi_i, b, t, mu_i, mu_j - mu_i))
    return samples


def train(net, mesh, pairs, epochs=10, batch=4, lr=1e-3, lr_end=1e-4, seed=0, log=None):
    """Adam on shuffled minibatches (seeded order), learning rate decayed
    geometrically from lr to lr_end.  Returns the mean loss per epoch."""
    rng = np.random.default_rng(seed)
    steps = epochs * ((len(pairs) + batch - 1) // batch)
    k = 0
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot, cnt = 0.0, 0
        for b0 in range(0, len(pairs), batch):
            idx = order[b0:b0 + batch]
            rate = lr * (lr_end / lr) ** (k / max(1, steps - 1))
            loss = net.train_step(mesh, [pairs[i][0] for i in idx], [pairs[i][1] for i in idx],
                                  [pairs[i][3] for i in idx], [pairs[i][4] for i in idx],
                                  [pairs[i][2] for i in idx], lr=rate)
            tot += loss * len(idx)
            cnt += len(idx)
            k += 1
        hist.append(tot / cnt)
        if log:
            log(f"[train] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
    return hist


class LearnedPredictor:
    """predictor(psi_m, psi_prev, mu_prev, mu_m, mu_next) for continuation_path:
    the network's correction of the secant start.  select="always" (default)
    uses the network's start unless it is not finite; select="residual" keeps
    the plain secant start when it has the smaller ||GL||_D at mu_next (the
    mesh's field must already be mu_next; continuation_path sets it).  The
    residual is a poor judge here: the network's start carries BF16-level
    high-frequency noise that the GL operator amplifies while Newton removes it
    in a step, so the network's start wins on Newton steps although its
    residual is larger.  Counts which start was used and records both
    residuals."""

    def __init__(self, net, mesh, select="always"):
        self.select = select
        import torch
        self.net, self.mesh = net, mesh
        self.out = None
        self.sec = None
        self.used = {"learned": 0, "secant": 0}
        self.residuals = []
        self.torch = torch

    def __call__(self, psi, prev, mu_prev, mu, mu_next):
        if self.out is None:
            self.out = self.torch.empty_like(psi)
            self.sec = self.torch.empty_like(psi)
        secant_base(self.mesh, psi, prev, mu_prev, mu, mu_next, self.sec)
        self.net.predict(self.mesh, psi, self.sec, mu, mu_next - mu, self.out)
        r_net = glnk.gl_residual(self.mesh, self.out)
        r_sec = glnk.gl_residual(self.mesh, self.sec)
        self.residuals.append((r_sec, r_net))
        bad = not np.isfinite(r_net)
        if bad or (self.select == "residual" and not r_net < r_sec):
            self.used["secant"] += 1
            return self.sec
        self.used["learned"] += 1
        return self.out


def init_params(levels, base, seed=0):
    return inputs.unet_init(glnk.unet_layer_shapes(levels, base), seed=seed, head_scale=0.0)
