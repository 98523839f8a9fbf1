"""Learned block ranks: training data from built operators, GPU training, slot sizing.

A far block's ACA rank is predicted from its geometry so that factor storage can be laid out
before ACA runs (HMX_RANK_LEARNED).  The network and its training run in libhmx's kernels; this
module only gathers (features, rank) pairs from operators built with plain adaptive ACA,
standardizes the features, calls the training entry point, and chooses the slot rule
r_alloc = ceil(alpha * r_hat) + beta so that a target fraction of the training blocks fit.
"""
from __future__ import annotations

import numpy as np

from . import hmx


def he_init(seed: int) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)) and zero biases, float32."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((64, 4)) * np.sqrt(2.0 / 4)
    w2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * np.sqrt(2.0 / 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3,
                           np.zeros(1)]).astype(np.float32)


def block_data(op: "hmx.Operator"):
    """(features (n, 4) float32, ranks (n,) int) of the low-rank far blocks of an operator."""
    feat = op.far_features()
    _, _, ranks = op.export_blocks()
    keep = ranks >= 0  # blocks stored dense carry no rank
    return feat[keep], ranks[keep].astype(np.int64)


class RankModel:
    def __init__(self, theta, norm, alpha=1.0, beta=0.0, history=None):
        self.theta = np.asarray(theta, np.float32)
        self.norm = np.asarray(norm, np.float32)
        self.alpha = float(alpha)
        self.beta = float(beta)
        self.history = history

    def install(self):
        """Make this the model used by builds with rank_model=RANK_LEARNED."""
        hmx.set_rank_model(self.theta, self.norm, self.alpha, self.beta)

    def predict_rank(self, feat):
        import torch
        f = torch.from_numpy(np.ascontiguousarray(feat, np.float32)).cuda()
        return np.expm1(hmx.mlp_predict(self.theta, self.norm, f).cpu().numpy().astype(np.float64))

    def save(self, path):
        np.savez(path, theta=self.theta, norm=self.norm, alpha=np.float32(self.alpha),
                 beta=np.float32(self.beta))

    @staticmethod
    def load(path):
        z = np.load(path, allow_pickle=False)
        return RankModel(z["theta"], z["norm"], float(z["alpha"]), float(z["beta"]))


def train(feat, ranks, epochs=60, batch=4096, lr=1e-3, seed=0, coverage=0.95, beta=2.0):
    """Train on (raw features, ranks); returns a RankModel with alpha chosen for `coverage`."""
    import torch
    feat = np.asarray(feat, np.float64)
    ranks = np.asarray(ranks, np.float64)
    mean = feat.mean(0)
    std = np.maximum(feat.std(0), 1e-6)
    norm = np.concatenate([mean, std]).astype(np.float32)
    perm = np.random.default_rng(seed).permutation(len(ranks))
    X = ((feat - mean) / std)[perm].astype(np.float32)
    y = np.log1p(ranks)[perm].astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    theta, hist = hmx.mlp_train(he_init(seed), Xd, yd, epochs=epochs, batch=batch, lr=lr)
    model = RankModel(theta, norm, 1.0, beta, hist)
    rhat = model.predict_rank(feat)
    ratio = (ranks - beta) / np.maximum(rhat, 1e-6)
    model.alpha = float(max(1.0, np.quantile(ratio, coverage)))
    return model
