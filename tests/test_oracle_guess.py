"""Pins of the FP64 oracle of the learned initial guess (features, network, Adam) against facts
that do not come from the oracle itself: central differences of the loss, special cases of the
network with a closed form, Adam's closed form under a constant gradient and its convergence on
a quadratic, brute-force image sums for the radial features, the isolated-atom case of the
bases, and rotation / permutation symmetry of features and bases.  CPU only."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from oracle import guess as G
from paper_2011_01207_amd import synth


def random_model(rng, scale=0.4):
    p = rng.standard_normal(G.NPARAM) * scale
    mean = rng.standard_normal(G.NFEAT) * 0.3
    inv = rng.uniform(0.5, 2.0, G.NFEAT)
    return np.concatenate([p, mean, inv])


def random_batch(rng, n=7):
    x = rng.standard_normal((n, G.NFEAT))
    b = rng.standard_normal((n, G.NBASIS, 3)) * 0.1
    t = rng.standard_normal((n, 3)) * 0.1
    return x, b, t


@pytest.mark.parametrize("kind", ["neumann", "delta"])
def test_gradient_matches_central_differences(kind):
    rng = np.random.default_rng(21)
    model = random_model(rng)
    x, b, t = random_batch(rng)
    off = G.OFFSETS[kind]
    _, g = G.loss_grad(model, x, b, t, offsets=off)
    h = 1e-6
    num = np.empty(G.NPARAM)
    for k in range(G.NPARAM):
        mp = model.copy()
        mm = model.copy()
        mp[k] += h
        mm[k] -= h
        num[k] = (G.loss(mp, x, b, t, offsets=off) - G.loss(mm, x, b, t, offsets=off)) / (2 * h)
    rel = np.linalg.norm(g - num) / np.linalg.norm(num)
    assert rel < 1e-6, rel
    # every block of the parameter vector carries gradient (no dead branch)
    off = 0
    for size in (64 * G.NFEAT, 64, 64 * 64, 64, 3 * 64, 3):
        blk = slice(off, off + size)
        assert np.linalg.norm(num[blk]) > 0
        assert np.linalg.norm(g[blk] - num[blk]) <= 1e-6 * np.linalg.norm(num[blk]) + 1e-12
        off += size


def test_loss_is_mean_squared_error_in_debye():
    rng = np.random.default_rng(3)
    model = random_model(rng)
    x, b, t = random_batch(rng, 5)
    mu0 = G.forward(model, x, b)
    # Debye^2 * mean over atoms of |mu0 - t|^2, computed component by component
    acc = 0.0
    for i in range(5):
        for c in range(3):
            acc += (4.80320 * (mu0[i, c] - t[i, c])) ** 2
    assert abs(G.loss(model, x, b, t) - acc / 5) < 1e-12 * acc


def test_untrained_network_returns_sum_of_bases():
    model = synth.guess_init_model(seed=7).astype(np.float64)
    rng = np.random.default_rng(4)
    x, b, _ = random_batch(rng)
    assert np.allclose(G.forward(model, x, b), b.sum(axis=1), atol=0, rtol=1e-15)


def test_untrained_delta_network_returns_the_reference():
    """With the delta offsets (1, 0, 0) and a zero last layer, mu0 is the first basis, the
    reference dipoles, exactly."""
    model = synth.guess_init_model(seed=7).astype(np.float64)
    rng = np.random.default_rng(14)
    x, b, _ = random_batch(rng)
    assert np.array_equal(G.forward(model, x, b, offsets=G.OFFSETS["delta"]), b[:, 0])


def test_delta_bases_special_cases():
    """The delta bases are (mu_ref, alpha (E - E_ref), alpha E): the second vanishes when the
    configuration's field equals the reference's, and the first is mu_ref whatever the field."""
    s = synth.tiny_cell(6, 12.0, seed=134, min_dist=1.0)
    rng = np.random.default_rng(15)
    e = rng.standard_normal((s.n, 3)) * 0.05
    mu_ref = rng.standard_normal((s.n, 3)) * 0.02
    b = G.bases_delta(s, e, mu_ref, e)
    assert np.array_equal(b[:, 0], mu_ref) and np.all(b[:, 1] == 0.0)
    for i in range(s.n):
        for c in range(3):
            assert b[i, 2, c] == s.alpha[i] * e[i, c]
    e_ref = e + rng.standard_normal((s.n, 3)) * 0.01
    b2 = G.bases_delta(s, e, mu_ref, e_ref)
    assert np.allclose(b2[:, 1], s.alpha[:, None] * (e - e_ref), rtol=1e-15, atol=0)
    # the cosine of the second and third basis is that of (E - E_ref) and E: alpha drops out
    x, _ = G.features_delta(s, e, mu_ref, e_ref)
    d = e - e_ref
    cos = np.sum(d * e, axis=1) / np.linalg.norm(d, axis=1) / np.linalg.norm(e, axis=1)
    assert np.allclose(x[:, 7], cos, rtol=1e-12)
    assert np.all(x[:, 8:] == 0.0)      # the delta kind leaves the radial sums out


def test_constant_last_layer():
    rng = np.random.default_rng(5)
    model = random_model(rng)
    w = G.unpack(model)
    c = np.array([0.5, -0.25, 2.0])
    m2 = G.pack(w["W1"], w["b1"], w["W2"], w["b2"], np.zeros((3, 64)), c, w["mean"], w["inv_std"])
    x, b, _ = random_batch(rng)
    expect = 1.5 * b[:, 0] + 0.75 * b[:, 1] + 3.0 * b[:, 2]
    assert np.allclose(G.forward(m2, x, b), expect, rtol=1e-14, atol=1e-16)


def test_silu_layers_single_unit():
    """One active hidden path written out by hand: x -> a1 = w x -> silu -> a2 = v silu(a1) -> silu
    -> y0 = u silu(a2); mu0 = (1 + y0) v0 + v1 + v2."""
    W1 = np.zeros((64, G.NFEAT))
    W2 = np.zeros((64, 64))
    W3 = np.zeros((3, 64))
    W1[5, 2] = 0.7
    W2[9, 5] = -1.3
    W3[0, 9] = 0.4
    model = G.pack(W1, np.zeros(64), W2, np.zeros(64), W3, np.zeros(3), np.zeros(G.NFEAT), np.ones(G.NFEAT))
    x = np.zeros((1, G.NFEAT))
    x[0, 2] = 1.1
    b = np.arange(9, dtype=float).reshape(1, 3, 3) * 0.01 + 0.02
    a1 = 0.7 * 1.1
    h1 = a1 / (1 + math.exp(-a1))
    a2 = -1.3 * h1
    h2 = a2 / (1 + math.exp(-a2))
    y0 = 0.4 * h2
    expect = (1 + y0) * b[0, 0] + b[0, 1] + b[0, 2]
    assert np.allclose(G.forward(model, x, b)[0], expect, rtol=1e-14)


def test_fit_norm_special_cases():
    x = np.zeros((4, G.NFEAT))
    x[:, 0] = [0.0, 2.0, 0.0, 2.0]        # mean 1, population std 1
    x[:, 1] = 0.39                         # constant: 1/std = 0
    x[:, 2] = [1.0, 1.0, 1.0, 5.0]        # mean 2, std sqrt(3)
    mean, inv = G.fit_norm(x)
    assert mean[0] == 1.0 and abs(inv[0] - 1.0) < 1e-15
    assert abs(mean[1] - 0.39) < 1e-15 and inv[1] == 0.0
    assert abs(mean[2] - 2.0) < 1e-15 and abs(inv[2] - 1 / math.sqrt(3.0)) < 1e-15


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2, so every
    step moves each parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    g = rng.standard_normal(G.NPARAM)
    g[:5] = [1e-3, -2.0, 0.0, 5e-9, -7.0]
    p0 = rng.standard_normal(G.NMODEL)
    p, m, v = p0.copy(), np.zeros(G.NPARAM), np.zeros(G.NPARAM)
    lr = 1e-2
    for t in range(1, 6):
        p, m, v = G.adam_step(p, m, v, t, g, lr)
    step = lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(p[:G.NPARAM], p0[:G.NPARAM] - 5 * step, rtol=1e-9, atol=1e-13)
    assert np.array_equal(p[G.NPARAM:], p0[G.NPARAM:])     # normalisation entries untouched


def test_adam_minimises_quadratic():
    rng = np.random.default_rng(8)
    target = rng.standard_normal(G.NPARAM)
    c = rng.uniform(0.5, 2.0, G.NPARAM)
    p, m, v = np.zeros(G.NMODEL), np.zeros(G.NPARAM), np.zeros(G.NPARAM)
    for t in range(1, 3001):
        grad = 2 * c * (p[:G.NPARAM] - target)
        p, m, v = G.adam_step(p, m, v, t, grad, 1e-2)
    assert np.max(np.abs(p[:G.NPARAM] - target)) < 1e-2


def brute_radial(s):
    """x8..x10 by an explicit loop over atoms and the 27 nearest periodic images."""
    out = np.zeros((s.n, 3))
    L = s.box[0]
    for i in range(s.n):
        for j in range(s.n):
            for nx in (-1, 0, 1):
                for ny in (-1, 0, 1):
                    for nz in (-1, 0, 1):
                        if i == j and nx == ny == nz == 0:
                            continue
                        d = s.pos[i] - s.pos[j] - L * np.array([nx, ny, nz])
                        r = math.sqrt(float(d @ d))
                        if r < s.cutoff:
                            for k, ck in enumerate((1.0, 2.0, 3.0)):
                                out[i, k] += math.exp(-((r - ck) / 0.6) ** 2)
    return out


def test_radial_features_brute_force_images():
    s = synth.tiny_cell(9, 14.5, seed=131, min_dist=0.9)
    assert np.allclose(G.radial_sums(s), brute_radial(s), rtol=1e-13, atol=1e-14)


def test_isolated_atom_bases():
    """A single atom with no neighbour inside the cutoff: R vanishes, so v1 = alpha c v0 and
    v2 = (alpha c)^2 v0, with c the Ewald self coefficient."""
    s = synth.tiny_cell(1, 16.0, seed=132)
    e = np.array([[0.03, -0.02, 0.05]])
    b = G.bases(s, e)
    ac = s.alpha[0] * 4 * s.ewald_alpha ** 3 / (3 * math.sqrt(math.pi))
    assert np.allclose(b[0, 0], s.alpha[0] * e[0], rtol=1e-15)
    assert np.allclose(b[0, 1], ac * b[0, 0], rtol=1e-14)
    assert np.allclose(b[0, 2], ac * ac * b[0, 0], rtol=1e-14)
    x, _ = G.features(s, e)
    assert np.allclose(x[0, 5:8], 1.0, rtol=1e-14) and np.all(x[0, 8:] == 0.0)


def test_features_rotation_and_permutation_symmetry():
    """A 90 degree rotation about z maps the periodic cube onto itself: features are
    unchanged, bases rotate with the field.  Relabelling atoms permutes both."""
    s = synth.tiny_cell(12, 15.0, seed=133, min_dist=1.0)
    rng = np.random.default_rng(9)
    e = rng.standard_normal((s.n, 3)) * 0.05
    x, b = G.features(s, e)
    rot = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    sr = dataclasses.replace(s, pos=np.mod(s.pos @ rot.T, s.box))
    xr, br = G.features(sr, e @ rot.T)
    assert np.allclose(xr, x, rtol=1e-11, atol=1e-12)
    assert np.allclose(br, b @ rot.T, rtol=1e-11, atol=1e-14)
    perm = rng.permutation(s.n)
    sp = dataclasses.replace(s, pos=s.pos[perm], alpha=s.alpha[perm], thole=s.thole[perm])
    xp, bp = G.features(sp, e[perm])
    assert np.allclose(xp, x[perm], rtol=1e-12, atol=1e-14)
    assert np.allclose(bp, b[perm], rtol=1e-12, atol=1e-16)
    # the delta bases and features: invariant and equivariant in the same way
    mu_ref = rng.standard_normal((s.n, 3)) * 0.02
    e_ref = e + rng.standard_normal((s.n, 3)) * 0.01
    xd, bd = G.features_delta(s, e, mu_ref, e_ref)
    xdr, bdr = G.features_delta(sr, e @ rot.T, mu_ref @ rot.T, e_ref @ rot.T)
    assert np.allclose(xdr, xd, rtol=1e-11, atol=1e-12)
    assert np.allclose(bdr, bd @ rot.T, rtol=1e-11, atol=1e-14)


def test_sampled_features_equal_full():
    s = synth.water648()
    rng = np.random.default_rng(10)
    e = rng.standard_normal((s.n, 3)) * 0.05
    x, b = G.features(s, e)
    idx = np.sort(rng.choice(s.n, 40, replace=False))
    xs, bs = G.features(s, e, idx=idx)
    assert np.allclose(xs, x[idx], rtol=1e-12, atol=1e-14)
    assert np.allclose(bs, b[idx], rtol=1e-12, atol=1e-16)


@pytest.mark.slow
def test_oracle_training_reduces_error_and_iterations():
    """Sanity of the whole recipe in FP64: a few hundred Adam steps on a short trajectory of the
    648-atom box lower the loss, and the trained guess needs fewer PCG iterations than zero."""
    base = synth.water648()
    frames = list(synth.trajectory(base, 8, 0.02, seed=104))
    xs, bs, ys, data = [], [], [], []
    for p in frames:
        s = dataclasses.replace(base, pos=p)
        e = O.perm_field(s, "spme")
        mu, _, _ = O.pcg(s, e, "spme", tol_debye=1e-9)
        x, b = G.features(s, e)
        data.append((s, e, mu, x, b))
    X = np.concatenate([d[3] for d in data[:6]])
    B = np.concatenate([d[4] for d in data[:6]])
    Y = np.concatenate([d[2] for d in data[:6]])
    model = synth.guess_init_model(seed=7).astype(np.float64)
    mean, inv = G.fit_norm(X)
    model[G.NPARAM:G.NPARAM + G.NFEAT] = mean
    model[G.NPARAM + G.NFEAT:] = inv
    l0 = G.loss(model, X, B, Y)
    m, v = np.zeros(G.NPARAM), np.zeros(G.NPARAM)
    for t in range(1, 301):
        _, g = G.loss_grad(model, X, B, Y)
        model, m, v = G.adam_step(model, m, v, t, g, 1e-3)
    assert G.loss(model, X, B, Y) < 0.7 * l0
    s, e, mu, x, b = data[7]
    _, it_zero, _ = O.pcg(s, e, "spme", tol_debye=1e-5)
    _, it_learn, _ = O.pcg(s, e, "spme", tol_debye=1e-5, mu0=G.forward(model, x, b))
    assert it_learn < it_zero
