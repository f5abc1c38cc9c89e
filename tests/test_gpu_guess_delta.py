"""GPU parity of the learned guess's delta kind (a configuration that follows a solved one:
bases mu_ref, alpha (E - E_ref) and alpha E, offsets (1, 0, 0)) against the FP64 oracle, the
versioned checkpoint of the learned guess, and what the trained delta network gains over the
previous-step guess on held-out configurations of a trajectory."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from oracle import guess as G
from paper_2011_01207_amd import amoeba, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_model(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    m = synth.guess_init_model(seed=seed).astype(np.float64)
    m[G.NPARAM - 3 * 64 - 3:G.NPARAM] = rng.standard_normal(3 * 64 + 3) * scale
    m[:G.NPARAM] += rng.standard_normal(G.NPARAM) * 0.05
    m[G.NPARAM:G.NPARAM + G.NFEAT] = rng.standard_normal(G.NFEAT) * 0.2
    m[G.NPARAM + G.NFEAT:] = rng.uniform(0.5, 2.0, G.NFEAT)
    return m.astype(np.float32)


@pytest.fixture(scope="module")
def pair_of_frames():
    """Two consecutive configurations of the 648-atom box: the oracle's E_perm and mu* of the
    first (the reference) and E_perm of the second."""
    base = synth.water648()
    p0, p1 = list(synth.trajectory(base, 2, 0.02, seed=111))
    s0, s1 = dataclasses.replace(base, pos=p0), dataclasses.replace(base, pos=p1)
    e0 = O.perm_field(s0, "spme")
    mu0, _, _ = O.pcg(s0, e0, "spme", tol_debye=1e-10)
    e1 = O.perm_field(s1, "spme")
    mu1, _, _ = O.pcg(s1, e1, "spme", tol_debye=1e-10)
    return base, s1, e0, mu0, e1, mu1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_delta_features_forward_and_predict_match_oracle(pair_of_frames, prec):
    base, s1, e0, mu0, e1, _ = pair_of_frames
    print(f"[gpu] delta-kind features water_648 {prec}", flush=True)
    x_ref, b_ref = G.features_delta(s1, e1, mu0, e0)
    model = random_model(80)
    ctx, t = amoeba.context_for(s1, precision=prec, device=DEV)
    try:
        ctx.guess_set_kind("delta")
        ctx.guess_set_model(model)
        ctx.guess_set_reference(torch.tensor(mu0, device=DEV), torch.tensor(e0, device=DEV))
        et = torch.tensor(e1, device=DEV)
        feat, basis = ctx.guess_features(t["pos"], et)
        x = feat.cpu().numpy().astype(np.float64)
        b = basis.cpu().numpy().astype(np.float64)
        # the bases are the inputs themselves (FP32 copies); the radial features as in the
        # Neumann kind
        for k in range(3):
            d = np.linalg.norm(b[:, k] - b_ref[:, k], axis=1)
            assert d.max() <= 2e-7 * np.abs(b_ref[:, k]).max() + 1e-12, k
        assert np.allclose(x[:, 0:2], x_ref[:, 0:2], rtol=1e-6)
        assert np.allclose(x[:, 2:5], x_ref[:, 2:5], rtol=2e-6, atol=1e-9)
        assert np.abs(x[:, 5:8] - x_ref[:, 5:8]).max() < 2e-5
        assert np.allclose(x[:, 8:11], x_ref[:, 8:11], rtol=2e-5, atol=1e-6)
        mu_f = ctx.guess_forward(feat, basis).double().cpu().numpy()
        mu_o = G.forward(model.astype(np.float64), x, b, offsets=G.OFFSETS["delta"])
        assert rel(mu_f, mu_o) < 1e-5
        mu_p = ctx.guess_predict(t["pos"], et).cpu().numpy()
        assert rel(mu_p, G.forward(model.astype(np.float64), x_ref, b_ref, offsets=G.OFFSETS["delta"])) < 2e-5
    finally:
        ctx.close()


def test_untrained_delta_start_is_the_previous_step_start(pair_of_frames):
    """With the untrained network the delta guess is mu_ref itself (to FP32 rounding): the
    learned start needs the previous-step start's iterations (+-1) and reaches the oracle's
    mu* at the tolerance."""
    base, s1, e0, mu0, e1, mu1 = pair_of_frames
    ctx, t = amoeba.context_for(s1, precision="fp64", device=DEV)
    try:
        ctx.guess_set_kind("delta")
        ctx.guess_set_model(synth.guess_init_model(seed=7))
        et = torch.tensor(e1, device=DEV)
        mref = torch.tensor(mu0, device=DEV)
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.polarize(t["pos"], et, guess_mode="learned", tol_debye=1e-5)
        assert ei.value.status == amoeba.AMOEBA_E_STATE      # no reference yet
        ctx.guess_set_reference(mref, torch.tensor(e0, device=DEV))
        mu_l, _, it_l, st = ctx.polarize(t["pos"], et, guess_mode="learned", tol_debye=1e-5)
        assert st == amoeba.AMOEBA_OK
        mu_g, _, it_g, st = ctx.polarize(t["pos"], et, mu_guess=mref, guess_mode="given", tol_debye=1e-5)
        assert st == amoeba.AMOEBA_OK
        print(f"  untrained delta start {it_l} iterations, previous-step start {it_g}", flush=True)
        assert abs(it_l - it_g) <= 1
        for mu in (mu_l, mu_g):
            assert O.rms_debye(mu.cpu().numpy() - mu1) <= 1e-5
        # a non-finite reference is reported by the call that uses it
        bad = torch.tensor(mu0, device=DEV)
        bad[3, 1] = float("nan")
        ctx.guess_set_reference(bad, torch.tensor(e0, device=DEV))
        for call in (lambda: ctx.polarize(t["pos"], et, guess_mode="learned", tol_debye=1e-5),
                     lambda: ctx.guess_predict(t["pos"], et), lambda: ctx.guess_features(t["pos"], et)):
            with pytest.raises(amoeba.AmoebaError) as ei:
                call()
            assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
        ctx.guess_set_reference(mref, torch.tensor(e0, device=DEV))
        mu_l2, _, it_l2, st = ctx.polarize(t["pos"], et, guess_mode="learned", tol_debye=1e-5)
        # FP64 LDS sums run in a varying order: equal to rounding
        assert st == amoeba.AMOEBA_OK and it_l2 == it_l
        assert O.rms_debye((mu_l2 - mu_l).cpu().numpy()) < 1e-9
        assert amoeba.lib().amoeba_guess_set_kind(ctx.h, 7) == amoeba.AMOEBA_E_INVALID
    finally:
        ctx.close()


def test_checkpoint_resumes_training_exactly():
    """Save after some Adam steps, load into a fresh context, take the same further steps in
    both: the models are bitwise equal, so the checkpoint holds the moments and the step count.
    Blobs of the wrong size, magic, version or shape, or with NaN, are rejected and change
    nothing."""
    rng = np.random.default_rng(85)
    rows = 3000
    x = torch.tensor(rng.standard_normal((rows, G.NFEAT)).astype(np.float32), device=DEV)
    b = torch.tensor((rng.standard_normal((rows, 3, 3)) * 0.1).astype(np.float32), device=DEV)
    y = torch.tensor((rng.standard_normal((rows, 3)) * 0.1).astype(np.float32), device=DEV)
    s = synth.water648()
    idx = [torch.tensor(rng.integers(0, rows, 512).astype(np.int32), device=DEV) for _ in range(8)]
    a, _ = amoeba.context_for(s, precision="mixed", device=DEV)
    c, _ = amoeba.context_for(s, precision="mixed", device=DEV)
    try:
        a.guess_set_kind("delta")
        a.guess_set_model(random_model(86))
        for k in range(4):
            a.guess_train_step(x, b, y, 1e-3, idx=idx[k])
        blob = a.guess_save()
        assert len(blob) == amoeba.GUESS_BLOB_BYTES
        c.guess_load(blob)
        assert np.array_equal(c.guess_get_model(), a.guess_get_model())
        for k in range(4, 8):
            la = a.guess_train_step(x, b, y, 1e-3, idx=idx[k])
            lc = c.guess_train_step(x, b, y, 1e-3, idx=idx[k])
            assert la == lc
        assert np.array_equal(c.guess_get_model(), a.guess_get_model())
        # the kind travels with the blob: c computes delta offsets (same loss as a)
        assert c.guess_gradient(x, b, y, n_batch=700)[0] == a.guess_gradient(x, b, y, n_batch=700)[0]
        before = c.guess_get_model()
        raw = bytearray(blob)
        cases = {"size": bytes(raw[:-4]),
                 "magic": bytes(b"XMGUESS\0" + raw[8:]),
                 "version": bytes(raw[:8] + (2).to_bytes(4, "little") + raw[12:]),
                 "shape": bytes(raw[:16] + (12).to_bytes(4, "little") + raw[20:])}
        nan = bytearray(blob)
        nan[48:52] = np.array([np.nan], dtype=np.float32).tobytes()
        for name, bad in cases.items():
            with pytest.raises(amoeba.AmoebaError) as ei:
                c.guess_load(bad)
            assert ei.value.status == amoeba.AMOEBA_E_INVALID, name
        with pytest.raises(amoeba.AmoebaError) as ei:
            c.guess_load(bytes(nan))
        assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
        assert np.array_equal(c.guess_get_model(), before)
    finally:
        a.close()
        c.close()


def solve(ctx, pos, e, mode, prev=None, tol=1e-5):
    mu, _, it, st = ctx.polarize(pos, e, mu_guess=prev, guess_mode=mode, tol_debye=tol)
    assert st == amoeba.AMOEBA_OK
    return mu, it


def test_trained_delta_guess_gains_over_the_previous_step():
    """A 3,000-atom water box, 26 configurations of cumulative 0.02 A steps: the solver's own
    converged dipoles of configurations 1-19 (each with its predecessor as the reference) train
    the delta network on the GPU; on configurations 20-25 the learned start needs fewer PCG
    iterations than the previous-step start on average, every start converges to the oracle-free
    true-residual test, and the learned start's error is below the previous step's."""
    base = synth.water_box(1000, 31.05, 32, 7, "water_3000", buffer=1.0)
    frames = [torch.tensor(p, device=DEV) for p in synth.trajectory(base, 26, 0.02, seed=204)]
    print("[gpu] delta-kind training water_3000 trajectory", flush=True)
    ctx, t = amoeba.context_for(base, precision="mixed", device=DEV)
    try:
        ctx.guess_set_kind("delta")
        ref = []
        for pos in frames:
            ctx.build_blocklist(pos)
            e = ctx.perm_field(pos, t["q"], t["dip"], t["quad"])
            mu, _ = solve(ctx, pos, e, "zero", tol=1e-7)
            ref.append((pos, e, mu.clone()))
        feats, bases, targets = [], [], []
        for k in range(1, 20):
            ctx.build_blocklist(ref[k][0])
            ctx.guess_set_reference(ref[k - 1][2], ref[k - 1][1])
            f, bb = ctx.guess_features(ref[k][0], ref[k][1])
            feats.append(f)
            bases.append(bb)
            targets.append(ref[k][2].float())
        feat, basis, target = torch.cat(feats), torch.cat(bases), torch.cat(targets)
        ctx.guess_set_model(synth.guess_init_model(seed=7))
        ctx.guess_fit_norm(feat)
        rng = np.random.default_rng(5)
        for k in range(1500):
            idx = torch.tensor(rng.integers(0, feat.shape[0], 8192).astype(np.int32), device=DEV)
            ctx.guess_train_step(feat, basis, target, 2e-3, idx=idx)
        its = {"given": [], "learned": [], "best": []}
        err_l, err_p = [], []
        for k in range(20, 26):
            pos, e, mu_ref = ref[k]
            prev_mu, prev_e = ref[k - 1][2], ref[k - 1][1]
            ctx.build_blocklist(pos)
            ctx.guess_set_reference(prev_mu, prev_e)
            mu0 = ctx.guess_predict(pos, e)
            err_l.append(O.rms_debye((mu0 - mu_ref).cpu().numpy()))
            err_p.append(O.rms_debye((prev_mu - mu_ref).cpu().numpy()))
            for mode in its:
                mu, it = solve(ctx, pos, e, mode, prev=prev_mu if mode != "learned" else None)
                its[mode].append(it)
                z = (t["alpha"][:, None] * (e - ctx.dipole_matvec(pos, mu))).cpu().numpy()
                assert O.rms_debye(z) < 1e-5
        mean = {k: float(np.mean(v)) for k, v in its.items()}
        print(f"  guess error learned {np.mean(err_l):.4e} D, previous step {np.mean(err_p):.4e} D; "
              f"mean iterations {mean}", flush=True)
        assert np.mean(err_l) < 0.8 * np.mean(err_p)
        assert mean["learned"] < mean["given"]
        assert mean["best"] <= mean["given"]
    finally:
        ctx.close()
