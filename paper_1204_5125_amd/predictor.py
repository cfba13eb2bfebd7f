"""Learned Newton start for the mu-continuation (spec extension of the
continuation in Sec. 4): training data from a seeded continuation sweep,
training of the library's U-Net with its own kernels, and a predictor that
falls back to the secant step whenever the secant start has the smaller
GL residual.

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
    start, todo = psi0, list(mus)
    while todo:
        recs, _, st = continuation.continuation_path(mesh, start, todo, keep=True, **kw)
        records += recs
        states += st
        if recs[-1]["status"] == 0:
            break
        todo = [m for m in todo if m > recs[-1]["mu"] + 1e-12]
        if states:
            start = states[-1][1]
    return records, states


def make_pairs(mesh, states, strides=(1, 2, 3)):
    """Training pairs (psi_i, aligned psi_j, mu_i, mu_j - mu_i) for j = i + s.
    The target is rotated by the global phase that aligns it with psi_i
    (gl_secant_predict with ratio -1 gives e^{i chi} target)."""
    import torch
    pairs = []
    for s in strides:
        for i in range(len(states) - s):
            mu_i, psi_i = states[i]
            mu_j, psi_j = states[i + s]
            t = torch.empty_like(psi_i)
            glnk.gl_secant_predict(mesh, psi_i, psi_j, -1.0, t)
            pairs.append((psi_i, t, mu_i, mu_j - mu_i))
    return pairs


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
            loss = net.train_step(mesh, [pairs[i][0] for i in idx], [pairs[i][2] for i in idx],
                                  [pairs[i][3] for i in idx], [pairs[i][1] for i in idx], lr=rate)
            tot += loss * len(idx)
            cnt += len(idx)
            k += 1
        hist.append(tot / cnt)
        if log:
            log(f"[train] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
    return hist


class LearnedPredictor:
    """predictor(psi_m, psi_prev, mu_prev, mu_m, mu_next) for continuation_path: the
    network's start, unless the secant start (when there is one) has the
    smaller ||GL||_D at mu_next.  The mesh's field must already be mu_next
    (continuation_path sets it).  Counts which start was used."""

    def __init__(self, net, mesh):
        import torch
        self.net, self.mesh = net, mesh
        self.out = None
        self.sec = None
        self.used = {"learned": 0, "secant": 0}
        self.torch = torch

    def __call__(self, psi, prev, mu_prev, mu, mu_next):
        if self.out is None:
            self.out = self.torch.empty_like(psi)
            self.sec = self.torch.empty_like(psi)
        dmu = mu_next - mu
        self.net.predict(self.mesh, psi, mu, dmu, self.out)
        r_net = glnk.gl_residual(self.mesh, self.out)
        if prev is not None:
            glnk.gl_secant_predict(self.mesh, psi, prev, dmu / (mu - mu_prev), self.sec)
            r_sec = glnk.gl_residual(self.mesh, self.sec)
            if r_sec < r_net:
                self.used["secant"] += 1
                return self.sec
        self.used["learned"] += 1
        return self.out


def init_params(levels, base, seed=0):
    return inputs.unet_init(glnk.unet_layer_shapes(levels, base), seed=seed, head_scale=0.0)
