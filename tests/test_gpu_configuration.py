"""amoeba_polarize_configuration: list update, permanent field and solve in one call, against
the three separate calls (bitwise in mixed precision: the same kernels on the same data) and
against the oracle, along a short trajectory, with each start and the error paths."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2011_01207_amd import amoeba, synth
from parity_util import assert_fields  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def walk(s, n, seed):
    rng = np.random.default_rng(seed)
    d = np.zeros_like(s.pos)
    out = []
    for _ in range(n):
        d += rng.normal(0.0, 0.02, s.pos.shape)
        out.append(np.mod(s.pos + d, s.box))
    return out


@pytest.mark.parametrize("mode", ["zero", "given", "learned"])
def test_matches_the_separate_calls_bitwise(mode):
    s = dataclasses.replace(synth.solvated_chain_small(), buffer=1.0, sc_s_d=None)
    frames = [torch.tensor(p, device=DEV) for p in walk(s, 4, 31)]
    print(f"[gpu] configuration call, {mode} start", flush=True)
    a, t = amoeba.context_for(s, precision="mixed", device=DEV)
    b, _ = amoeba.context_for(s, precision="mixed", device=DEV)
    if mode == "learned":
        for c in (a, b):
            c.guess_set_kind("delta")
            c.guess_set_model(synth.guess_init_model(seed=7))
    prev = None
    for k, pos in enumerate(frames):
        guess = None if mode == "zero" or prev is None else prev[0]
        gm = mode if prev is not None else "zero"
        if gm == "learned":
            for c in (a, b):
                c.guess_set_reference(*prev)
        ra = a.update_blocklist(pos)
        ea = a.perm_field(pos, t["q"], t["dip"], t["quad"])
        mu_a, epa, ita, sta = a.polarize(pos, ea, mu_guess=guess, guess_mode=gm, tol_debye=1e-6)
        eb = torch.empty_like(ea)
        mu_b, _, epb, itb, stb, rb = b.polarize_configuration(pos, t["q"], t["dip"], t["quad"], mu_guess=guess,
                                                               guess_mode=gm, tol_debye=1e-6, e_perm_out=eb)
        assert sta == stb == amoeba.AMOEBA_OK and ra == rb
        assert torch.equal(ea, eb), k
        assert torch.equal(mu_a, mu_b) and epa == epb and ita == itb, k
        assert a.info()["last_guess"] == b.info()["last_guess"]
        prev = (mu_b.clone(), eb.clone())
    # a step beyond buffer/2: both rebuild (the single call after computing the configuration
    # once on the stale list) and agree bitwise
    far = frames[-1].clone()
    far[5, 0] += 0.6
    assert a.update_blocklist(far)
    ea = a.perm_field(far, t["q"], t["dip"], t["quad"])
    mu_a, epa, ita, _ = a.polarize(far, ea, tol_debye=1e-6)
    eb = torch.empty_like(ea)
    mu_b, _, epb, itb, stb, rb = b.polarize_configuration(far, t["q"], t["dip"], t["quad"], tol_debye=1e-6,
                                                           e_perm_out=eb)
    assert rb and stb == amoeba.AMOEBA_OK
    assert torch.equal(ea, eb) and torch.equal(mu_a, mu_b) and epa == epb and ita == itb
    assert a.info()["n_pairs"] == b.info()["n_pairs"]
    a.close()
    b.close()


def test_fp64_against_the_oracle():
    s = dataclasses.replace(synth.water648(), buffer=1.0)
    pos = walk(s, 1, 33)[0]
    s1 = dataclasses.replace(s, pos=pos)
    ctx, t = amoeba.context_for(s, precision="fp64", device=DEV)
    e = torch.empty((s.n, 3), dtype=torch.float64, device=DEV)
    mu, _, ep, it, st, rebuilt = ctx.polarize_configuration(torch.tensor(pos, device=DEV), t["q"], t["dip"],
                                                            t["quad"], tol_debye=1e-9, e_perm_out=e)
    assert st == amoeba.AMOEBA_OK and not rebuilt
    e_ref = O.perm_field(s1, "spme")
    assert_fields(e.cpu().numpy(), e_ref, 1e-11, what="E_perm")
    mu_ref, _, _ = O.pcg(s1, e_ref, "spme", tol_debye=1e-10)
    assert O.rms_debye(mu.cpu().numpy() - mu_ref) < 1e-8
    assert abs(ep - O.e_pol(mu_ref, e_ref)) < 1e-8 * abs(ep)
    ctx.close()


def test_errors():
    s = synth.water648()
    bare = amoeba.Context(s.n, s.box, cutoff=s.cutoff, ewald_alpha=s.ewald_alpha, grid=s.grid, precision="mixed")
    tp = torch.tensor(s.pos, device=DEV)
    with pytest.raises(amoeba.AmoebaError) as e:                # no amoeba_set_atoms yet
        bare.polarize_configuration(tp, tp[:, 0].contiguous(), tp, torch.zeros((s.n, 6), dtype=torch.float64,
                                                                               device=DEV))
    assert e.value.status == amoeba.AMOEBA_E_STATE
    bare.close()
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    # an iteration budget too small: NOT_CONVERGED with the last iterate
    mu, _, _, it, st, _ = ctx.polarize_configuration(t["pos"], t["q"], t["dip"], t["quad"], tol_debye=1e-9,
                                                     max_iter=2)
    assert st == amoeba.AMOEBA_NOT_CONVERGED and it == 2 and torch.isfinite(mu).all()
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.polarize_configuration(t["pos"], t["q"], t["dip"], t["quad"], guess_mode="learned")
    assert e.value.status == amoeba.AMOEBA_E_STATE            # no model loaded
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.polarize_configuration(t["pos"], t["q"], t["dip"], t["quad"], guess_mode="given")
    assert e.value.status == amoeba.AMOEBA_E_INVALID          # GIVEN without mu_guess
    bad = t["quad"].clone()
    bad[3, 0] += 0.5                                          # trace 0.5: not traceless
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.polarize_configuration(t["pos"], t["q"], t["dip"], bad)
    assert e.value.status == amoeba.AMOEBA_E_INVALID and "traceless" in str(e.value)
    nanq = t["q"].clone()
    nanq[7] = float("nan")
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.polarize_configuration(t["pos"], nanq, t["dip"], t["quad"])
    assert e.value.status == amoeba.AMOEBA_E_NUMERIC
    nanpos = t["pos"].clone()
    nanpos[11, 1] = float("nan")
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.polarize_configuration(nanpos, t["q"], t["dip"], t["quad"])
    assert e.value.status == amoeba.AMOEBA_E_NUMERIC and "position" in str(e.value)
    # the context still works
    mu, _, _, _, st, _ = ctx.polarize_configuration(t["pos"], t["q"], t["dip"], t["quad"], tol_debye=1e-6)
    assert st == amoeba.AMOEBA_OK and torch.isfinite(mu).all()
    ctx.close()
