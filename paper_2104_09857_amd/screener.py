"""Training driver of the learned block screener (orchestration only).

Samples are (features, log10 ||chi_{cc'}(tau)||) of the upper output blocks
(c <= c') of exact chi runs; features and targets come from
gw_chi_block_features / gw_chi_block_lognorms, the network is trained by
gw_mlp_train_step (forward, backprop and Adam on the GPU) and evaluated by
gw_mlp_forward.  Inputs and targets are standardized for training; the
scales are folded into the first and last layer afterwards so that
gw_contract_chi can apply the network to raw features.
"""
from __future__ import annotations

import numpy as np

from . import gw

N_FEATURES = 6
HIDDEN = 64


def _he_init(seed):
    rng = np.random.default_rng(seed)
    F, H = N_FEATURES, HIDDEN
    w1 = rng.standard_normal((H, F)) * np.sqrt(2.0 / F)
    w2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H)
    w3 = rng.standard_normal((1, H)) * np.sqrt(1.0 / H)
    return pack(w1, np.zeros(H), w2, np.zeros(H), w3, np.zeros(1))


def pack(w1, b1, w2, b2, w3, b3):
    return np.concatenate([w1.ravel(), b1, w2.ravel(), b2, w3.ravel(), b3]).astype(np.float64)


def unpack(p):
    F, H = N_FEATURES, HIDDEN
    o = 0
    w1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    w2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H].reshape(1, H); o += H
    b3 = p[o:o + 1]
    return w1, b1, w2, b2, w3, b3


def samples(sys, d_occ, d_vir, chi, tau, filter_eps):
    """(X [n, 6], t [n]) device tensors for the upper blocks of every tau.

    chi should be the exact contraction without the output filter
    (contract_chi(..., keep_small_blocks=True)): its block norms are
    continuous through the threshold, whereas the filtered output jumps from
    just above the threshold to zero, a cliff the regression cannot follow
    (blocks just above it are then under-predicted by the depth of the
    target floor)."""
    import torch
    feat = gw.chi_block_features(sys, d_occ, d_vir, tau, filter_eps)
    lgn = gw.chi_block_lognorms(sys, chi)
    na = sys.c.n_atoms
    iu = torch.triu_indices(na, na, device=feat.device)
    X = feat[:, iu[0], iu[1], :].reshape(-1, N_FEATURES).contiguous()
    t = lgn[:, iu[0], iu[1]].reshape(-1).contiguous()
    return X, t


class BlockScreener:
    def __init__(self, seed=0, params=None):
        self.seed = seed
        self.params = _he_init(seed) if params is None else np.asarray(params, dtype=np.float64)
        self.x_mean = np.zeros(N_FEATURES)
        self.x_std = np.ones(N_FEATURES)
        self.t_mean, self.t_std = 0.0, 1.0
        self.net = None          # gw.Mlp on raw features (folded)
        self.margin = 1.0        # safety band in decades (see calibrate)

    def fit(self, X, t, filter_eps=None, floor_decades=3.0, steps=2000, batch=4096, lr=2e-3,
            alpha=8.0, log_every=200):
        """Train on device tensors X [n, F], t [n]; returns the loss history.

        With filter_eps given, targets are clipped from below at
        log10(filter_eps) - floor_decades: only the side of the threshold
        matters, and blocks that the exact run zeroes (log10 norm -30) would
        otherwise put a cliff into the regression target."""
        import torch
        if filter_eps is not None:
            t = torch.clamp(t, min=float(np.log10(filter_eps)) - floor_decades)
        self.x_mean = X.double().mean(0).cpu().numpy()
        self.x_std = X.double().std(0).cpu().numpy() + 1e-6
        self.t_mean = float(t.double().mean())
        self.t_std = float(t.double().std()) + 1e-6
        xm = torch.as_tensor(self.x_mean, dtype=torch.float32, device=X.device)
        xs = torch.as_tensor(self.x_std, dtype=torch.float32, device=X.device)
        Xn = ((X - xm) / xs).contiguous()
        tn = ((t - self.t_mean) / self.t_std).contiguous()
        net = gw.Mlp(N_FEATURES, HIDDEN, self.params)
        gen = torch.Generator(device=X.device)
        gen.manual_seed(self.seed)
        hist = []
        n = Xn.shape[0]
        for step in range(steps):
            idx = torch.randint(0, n, (min(batch, n),), device=X.device, generator=gen)
            loss = net.train_step(Xn[idx].contiguous(), tn[idx].contiguous(), alpha, lr)
            if step % log_every == 0 or step == steps - 1:
                hist.append((step, float(loss.item())))
        self.params = net.params.double().cpu().numpy()
        self.net = gw.Mlp(N_FEATURES, HIDDEN, self.folded())
        return hist

    def calibrate(self, X, t, filter_eps, safety=0.5):
        """Safety band (decades) from held-out samples: the largest amount by
        which the network under-predicts a block that the filter keeps
        (true log10 norm >= log10 filter_eps), plus `safety`."""
        import torch
        pred = self.predict(X)
        thr = float(np.log10(filter_eps))
        sel = t >= thr
        worst = float((thr - pred[sel]).max()) if bool(sel.any()) else 0.0
        self.margin = max(0.0, worst) + safety
        return self.margin

    def folded(self):
        """Parameters acting on raw features and returning raw log10 norms."""
        w1, b1, w2, b2, w3, b3 = unpack(self.params)
        w1f = w1 / self.x_std[None, :]
        b1f = b1 - w1f @ self.x_mean
        w3f = w3 * self.t_std
        b3f = b3 * self.t_std + self.t_mean
        return pack(w1f, b1f, w2, b2, w3f, b3f)

    def predict(self, X):
        if self.net is None:
            self.net = gw.Mlp(N_FEATURES, HIDDEN, self.folded())
        return self.net.forward(X, fp16=True)

    def save(self, path):
        np.savez(path, params=self.params, x_mean=self.x_mean, x_std=self.x_std,
                 t_mean=self.t_mean, t_std=self.t_std, seed=self.seed, margin=self.margin)

    @classmethod
    def load(cls, path):
        d = np.load(path)
        s = cls(int(d["seed"]), d["params"])
        s.x_mean, s.x_std = d["x_mean"], d["x_std"]
        s.t_mean, s.t_std = float(d["t_mean"]), float(d["t_std"])
        s.margin = float(d["margin"])
        return s
