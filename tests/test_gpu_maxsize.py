"""Full-size GPU parity on the two largest workloads: 96,000 waters (288,000 atoms, 142.3 A box,
grid 144^3) and 288,000 waters (864,000 atoms, 205.0 A box, grid 216^3), both with the 2 A list
buffer.  As on the benchmark box, the oracle computes sampled atoms one by one (real space
exactly, the reciprocal field from its full SPME grid), and the solve is checked through the
oracle's own residual of the GPU solution at those atoms."""
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
SYSTEMS = {"water_288000": synth.water288k, "water_864000": synth.water864k}




@pytest.fixture(scope="module", params=list(SYSTEMS))
def big(request):
    s = SYSTEMS[request.param]()
    idx = np.sort(np.random.default_rng(13).choice(s.n, 256, replace=False))
    print(f"[gpu] oracle references for {s.name} (sampled)", flush=True)
    mu = np.random.default_rng(14).standard_normal((s.n, 3)) * 0.05
    return s, idx, {"mu": mu, "matvec": O.matvec(s, mu, "spme", idx=idx),
                    "perm": O.perm_field(s, "spme", idx=idx)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sampled_fields_and_solve(big, prec):
    s, idx, ref = big
    print(f"[gpu] {s.name} {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        assert_fields(e.cpu().numpy()[idx], ref["perm"], (1e-11 if prec == "fp64" else 3e-5))
        q = ctx.dipole_matvec(t["pos"], torch.tensor(ref["mu"], device=DEV)).cpu().numpy()[idx]
        assert_fields(q, ref["matvec"], (1e-12 if prec == "fp64" else 3e-6))
        mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-5)
        assert st == amoeba.AMOEBA_OK and it > 0
        r = ref["perm"] - O.matvec(s, mu.cpu().numpy(), "spme", idx=idx)
        assert O.rms_debye(s.alpha[idx][:, None] * r) < 2.5e-5
    finally:
        ctx.close()


def test_mixed_matches_fp64(big):
    s, _, _ = big
    res = {}
    for prec in ("fp64", "mixed"):
        ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
        try:
            e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
            mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-7)
            assert st == amoeba.AMOEBA_OK
            res[prec] = (mu.cpu().numpy(), ep, ctx.info()["n_pairs"])
        finally:
            ctx.close()
    print(f"[gpu] {s.name}: {res['fp64'][2]} pairs, mixed vs FP64 "
          f"{O.rms_debye(res['mixed'][0] - res['fp64'][0]):.2e} D", flush=True)
    assert O.rms_debye(res["mixed"][0] - res["fp64"][0]) < 1e-5
    assert abs(res["mixed"][1] - res["fp64"][1]) < 1e-5 * abs(res["fp64"][1])
    assert res["mixed"][2] == res["fp64"][2] > 0
