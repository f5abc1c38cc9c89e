"""FP64 oracle of the learned initial guess for the induced-dipole solve.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's CPU-baseline
leg import this module.  It shares no code with the GPU library.

The paper solves the dipoles by PCG from a plain starting point; the learned guess is this
build's addition (a per-atom network over neighbour-list environment features predicting the
PCG starting point).  Everything here is the definition written out in plain NumPy:

Equivariant bases (e*A), with R the real-space Thole-damped Ewald dipole field over the
in-cutoff pairs and c = 4 beta^3 / (3 sqrt(pi)) the Ewald self coefficient:
    v0 = alpha E_perm,   v1 = alpha (R[v0] + c v0),   v2 = alpha (R[v1] + c v1)
(the first three terms of the Neumann series of (alpha^-1 - T)^-1 E_perm with the
reciprocal-space part left out).

Invariant features (NFEAT = 11):
    x0 = alpha, x1 = Thole a, x2..x4 = Debye * |v_k|,
    x5, x6, x7 = cos(v0, v1), cos(v0, v2), cos(v1, v2) with cos(a, b) = a.b / sqrt(|a|^2 |b|^2 + 1e-20),
    x8..x10 = sum over in-cutoff neighbours j of exp(-((r_ij - c_k) / 0.6)^2), c_k = 1, 2, 3 A.

Bases of the second kind, the "delta" guess for a configuration that follows a solved one
(mu_ref its converged dipoles, E_ref its permanent field):
    v0 = mu_ref,   v1 = alpha (E_perm - E_ref),   v2 = alpha E_perm
with the same invariant features computed from them, except x8..x10 (the radial sums), which
this kind leaves at zero.

Network: xh = (x - mean) * inv_std; h1 = silu(W1 xh + b1); h2 = silu(W2 h1 + b2);
y = W3 h2 + b3; mu0 = sum_k (s_k + y_k) v_k with the fixed offsets s = (1, 1, 1) for the
Neumann bases (an untrained network returns their sum) and s = (1, 0, 0) for the delta bases
(an untrained network returns mu_ref).  silu(a) = a / (1 + exp(-a)).
Loss over a batch of n atoms: L = Debye^2 / n * sum_i |mu0_i - mu*_i|^2 (D^2).
Optimiser: Adam (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and the bias
corrections of the published algorithm.

Parameter vector (float, NPARAM = 64*11 + 64 + 64*64 + 64 + 3*64 + 3 = 5123), row-major:
W1[64][11], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]; the model vector appends
mean[11] and inv_std[11] (NMODEL = 5145).
"""
from __future__ import annotations

import math

import numpy as np

from . import ref as O

NFEAT = 11
NBASIS = 3
HIDDEN = 64
NPARAM = HIDDEN * NFEAT + HIDDEN + HIDDEN * HIDDEN + HIDDEN + NBASIS * HIDDEN + NBASIS
NMODEL = NPARAM + 2 * NFEAT
RADIAL_CENTERS = (1.0, 2.0, 3.0)
RADIAL_WIDTH = 0.6
COS_EPS = 1e-20
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
OFFSETS = {"neumann": (1.0, 1.0, 1.0), "delta": (1.0, 0.0, 0.0)}


# ----------------------------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------------------------

def _min_image(d, box):
    return d - box * np.rint(d / box)


def neighbour_distances(s, idx):
    """Minimum-image distances from atoms idx to every atom, and the in-cutoff mask
    (0 < r < rc)."""
    d = _min_image(s.pos[idx][:, None, :] - s.pos[None, :, :], np.asarray(s.box))
    r = np.sqrt(np.sum(d * d, axis=2))
    m = (r < s.cutoff) & (np.arange(s.n)[None, :] != np.asarray(idx)[:, None])
    return r, m


def radial_sums(s, idx=None):
    """x8..x10: Gaussian-weighted neighbour counts over the in-cutoff pairs."""
    idx = np.arange(s.n) if idx is None else np.asarray(idx)
    out = np.zeros((len(idx), len(RADIAL_CENTERS)))
    for b0 in range(0, len(idx), 512):
        r, m = neighbour_distances(s, idx[b0:b0 + 512])
        for k, c in enumerate(RADIAL_CENTERS):
            out[b0:b0 + 512, k] = np.sum(np.where(m, np.exp(-((r - c) / RADIAL_WIDTH) ** 2), 0.0), axis=1)
    return out


def bases(s, e_perm, idx=None):
    """(v0, v1, v2) at atoms idx (all if None), shape [n][3][3].  For a sample, v1 is evaluated
    on the sampled atoms and their in-cutoff neighbours only (all that v2 at the sample needs)."""
    alpha = np.asarray(s.alpha, dtype=np.float64)[:, None]
    c = O.self_coeff(s.ewald_alpha)
    e = np.asarray(e_perm, dtype=np.float64)
    v0 = alpha * e
    if idx is None:
        v1 = alpha * (O.real_mutual(s, v0) + c * v0)
        v2 = alpha * (O.real_mutual(s, v1) + c * v1)
        return np.stack([v0, v1, v2], axis=1)
    idx = np.asarray(idx)
    near = set(idx.tolist())
    for b0 in range(0, len(idx), 512):
        _, m = neighbour_distances(s, idx[b0:b0 + 512])
        near.update(np.nonzero(m.any(axis=0))[0].tolist())
    u = np.array(sorted(near), dtype=np.int64)
    v1 = np.zeros_like(v0)
    v1[u] = alpha[u] * (O.real_mutual(s, v0, idx=u) + c * v0[u])
    v2 = alpha[idx] * (O.real_mutual(s, v1, idx=idx) + c * v1[idx])
    return np.stack([v0[idx], v1[idx], v2], axis=1)


def bases_delta(s, e_perm, mu_ref, e_ref, idx=None):
    """(mu_ref, alpha (E - E_ref), alpha E) at atoms idx (all if None), shape [n][3][3]."""
    idx = np.arange(s.n) if idx is None else np.asarray(idx)
    alpha = np.asarray(s.alpha, dtype=np.float64)[idx][:, None]
    e = np.asarray(e_perm, dtype=np.float64)[idx]
    return np.stack([np.asarray(mu_ref, dtype=np.float64)[idx],
                     alpha * (e - np.asarray(e_ref, dtype=np.float64)[idx]), alpha * e], axis=1)


def features_from(s, basis, radial, idx=None):
    idx = np.arange(s.n) if idx is None else np.asarray(idx)
    nrm = np.sqrt(np.sum(basis * basis, axis=2))            # [n][3]

    def cos(a, b):
        return np.sum(basis[:, a] * basis[:, b], axis=1) / np.sqrt(nrm[:, a] ** 2 * nrm[:, b] ** 2 + COS_EPS)

    x = np.empty((len(idx), NFEAT))
    x[:, 0] = np.asarray(s.alpha)[idx]
    x[:, 1] = np.asarray(s.thole)[idx]
    x[:, 2:5] = O.DEBYE * nrm
    x[:, 5] = cos(0, 1)
    x[:, 6] = cos(0, 2)
    x[:, 7] = cos(1, 2)
    x[:, 8:11] = radial
    return x


def features(s, e_perm, idx=None):
    """(x [n][NFEAT], basis [n][3][3]) at atoms idx (all if None)."""
    b = bases(s, e_perm, idx)
    return features_from(s, b, radial_sums(s, idx), idx), b


def features_delta(s, e_perm, mu_ref, e_ref, idx=None):
    """(x [n][NFEAT], basis [n][3][3]) of the delta bases at atoms idx (all if None)."""
    b = bases_delta(s, e_perm, mu_ref, e_ref, idx)
    n = s.n if idx is None else len(idx)
    return features_from(s, b, np.zeros((n, len(RADIAL_CENTERS))), idx), b


# ----------------------------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------------------------

def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (HIDDEN, NFEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
                        ("W3", (NBASIS, HIDDEN)), ("b3", (NBASIS,))):
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    if p.size >= NMODEL:
        out["mean"] = p[NPARAM:NPARAM + NFEAT]
        out["inv_std"] = p[NPARAM + NFEAT:NMODEL]
    return out


def pack(W1, b1, W2, b2, W3, b3, mean=None, inv_std=None):
    parts = [np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(W3), np.ravel(b3)]
    if mean is not None:
        parts += [np.ravel(mean), np.ravel(inv_std)]
    return np.concatenate(parts).astype(np.float64)


def fit_norm(x):
    """Per-feature mean and 1/std (population) over the samples; 1/std = 0 where std <= 1e-6."""
    x = np.asarray(x, dtype=np.float64)
    mean = np.mean(x, axis=0)
    std = np.sqrt(np.mean((x - mean) ** 2, axis=0))
    inv = np.where(std > 1e-6, 1.0 / np.where(std > 1e-6, std, 1.0), 0.0)
    return mean, inv


def _sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def forward(model, x, basis, return_cache=False, offsets=OFFSETS["neumann"]):
    """mu0 [n][3] for features x [n][NFEAT] and bases [n][3][3]."""
    w = unpack(model)
    xh = (np.asarray(x, dtype=np.float64) - w["mean"]) * w["inv_std"]
    a1 = xh @ w["W1"].T + w["b1"]
    h1 = a1 * _sigmoid(a1)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = a2 * _sigmoid(a2)
    y = h2 @ w["W3"].T + w["b3"]
    mu0 = np.sum((np.asarray(offsets, dtype=np.float64) + y)[:, :, None] * np.asarray(basis, dtype=np.float64),
                 axis=1)
    if return_cache:
        return mu0, (xh, a1, h1, a2, h2, y)
    return mu0


def loss_grad(model, x, basis, target, offsets=OFFSETS["neumann"]):
    """(L, dL/dparams [NPARAM]) by backpropagation through the network above."""
    w = unpack(model)
    basis = np.asarray(basis, dtype=np.float64)
    n = x.shape[0]
    mu0, (xh, a1, h1, a2, h2, y) = forward(model, x, basis, return_cache=True, offsets=offsets)
    diff = mu0 - np.asarray(target, dtype=np.float64)
    dd = O.DEBYE ** 2
    loss = dd / n * float(np.sum(diff * diff))
    g_mu = 2.0 * dd / n * diff                                  # dL/dmu0
    d3 = np.einsum("nc,nkc->nk", g_mu, basis)                   # dL/dy
    dW3 = d3.T @ h2
    db3 = d3.sum(axis=0)
    s2 = _sigmoid(a2)
    d2 = (d3 @ w["W3"]) * (s2 * (1.0 + a2 * (1.0 - s2)))        # silu'(a) = s (1 + a (1 - s))
    dW2 = d2.T @ h1
    db2 = d2.sum(axis=0)
    s1 = _sigmoid(a1)
    d1 = (d2 @ w["W2"]) * (s1 * (1.0 + a1 * (1.0 - s1)))
    dW1 = d1.T @ xh
    db1 = d1.sum(axis=0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


def loss(model, x, basis, target, offsets=OFFSETS["neumann"]):
    mu0 = forward(model, x, basis, offsets=offsets)
    return O.DEBYE ** 2 / x.shape[0] * float(np.sum((mu0 - np.asarray(target)) ** 2))


def adam_step(params, m, v, t, grad, lr):
    """One Adam update of the first NPARAM entries; t is the 1-based step number.  Returns the
    new (params, m, v)."""
    params = np.array(params, dtype=np.float64)
    m = ADAM_B1 * np.asarray(m) + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * np.asarray(v) + (1.0 - ADAM_B2) * grad * grad
    mhat = m / (1.0 - ADAM_B1 ** t)
    vhat = v / (1.0 - ADAM_B2 ** t)
    params[:NPARAM] -= lr * mhat / (np.sqrt(vhat) + ADAM_EPS)
    return params, m, v
