"""Full-size GPU parity on the benchmark workload (96,000-atom water box, the launch
configuration bench.py times), checked on sampled atoms the oracle computes one by one and
through properties that hold at any size (the oracle's residual of the GPU solution)."""
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




@pytest.fixture(scope="module")
def c2():
    s = synth.water96k()
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(s.n, 256, replace=False))
    return s, idx


@pytest.fixture(scope="module")
def c2_ref(c2):
    s, idx = c2
    print("[gpu] oracle references for water_96000 (sampled)", flush=True)
    mu = np.random.default_rng(12).standard_normal((s.n, 3)) * 0.05
    return {"mu": mu, "matvec": O.matvec(s, mu, "spme", idx=idx), "perm": O.perm_field(s, "spme", idx=idx)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_water96k_fields_and_solve(c2, c2_ref, prec):
    s, idx = c2
    print(f"[gpu] water_96000 {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    assert_fields(e.cpu().numpy()[idx], c2_ref["perm"], (1e-11 if prec == "fp64" else 3e-5))
    q = ctx.dipole_matvec(t["pos"], torch.tensor(c2_ref["mu"], device=DEV)).cpu().numpy()[idx]
    assert_fields(q, c2_ref["matvec"], (1e-12 if prec == "fp64" else 3e-6))
    # solve to 1e-5 D; the oracle's own residual of the GPU solution at the sampled atoms
    mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-5)
    assert st == amoeba.AMOEBA_OK and it > 0
    mu_np = mu.cpu().numpy()
    r = c2_ref["perm"] - O.matvec(s, mu_np, "spme", idx=idx)
    z = s.alpha[idx][:, None] * r
    assert O.rms_debye(z) < 2.5e-5
    ctx.close()


def test_water96k_mixed_matches_fp64_and_pair_count(c2):
    s, idx = c2
    res = {}
    for prec in ("fp64", "mixed"):
        ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-7)
        assert st == amoeba.AMOEBA_OK
        res[prec] = (mu.cpu().numpy(), ep, ctx.info()["n_pairs"])
        ctx.close()
    assert O.rms_debye(res["mixed"][0] - res["fp64"][0]) < 1e-5
    assert abs(res["mixed"][1] - res["fp64"][1]) < 1e-5 * abs(res["fp64"][1])
    assert res["mixed"][2] == res["fp64"][2] == O.count_pairs(s)


@pytest.fixture(scope="module")
def subcell864():
    """The periodic subcell of the 864,000-atom box (whole waters in 11 lattice spacings, grid
    36^3): small enough for the oracle's full SPME solve."""
    s = synth.subcell(synth.water864k())
    print(f"[gpu] oracle solve of the {s.n}-atom subcell", flush=True)
    e = O.perm_field(s, "spme")
    mu, _, _ = O.pcg(s, e, "spme", tol_debye=1e-10)
    return s, e, mu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_subcell_of_864k_box_dipoles_and_energy(subcell864, prec):
    """E_perm, mu and E_pol of the GPU solver against the oracle's exact SPME solution."""
    s, e_ref, mu_ref = subcell864
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    assert_fields(e.cpu().numpy(), e_ref, (1e-11 if prec == "fp64" else 3e-5))
    tol = 1e-9 if prec == "fp64" else 1e-6
    mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=tol)
    assert st == amoeba.AMOEBA_OK
    err = O.rms_debye(mu.cpu().numpy() - mu_ref)
    ep_ref = O.e_pol(mu_ref, e_ref)
    print(f"[gpu] subcell {prec}: {it} it, mu rms err {err:.2e} D, E_pol rel err {abs(ep - ep_ref) / abs(ep_ref):.2e}",
          flush=True)
    assert err < (5e-9 if prec == "fp64" else 5e-6)
    assert abs(ep - ep_ref) < (1e-9 if prec == "fp64" else 1e-6) * abs(ep_ref)
    ctx.close()
