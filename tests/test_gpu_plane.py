"""GPU parity of the plane path of the reciprocal dipole field (x-planes of the PME grid in LDS:
fused spread and y-z FFT, x-line FFT with the influence function, fused inverse y-z FFT and
interpolation) against the FP64 oracle's smooth PME and against the brick / rocFFT path of
the same context, on grids with odd edges, radices 2 to 7 and non-cubic shapes."""
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
TOL = {"fp64": 1e-11, "mixed": 2e-5}
# both paths on one context: same arithmetic up to summation order and FFT algorithm
TOL_PATHS = {"fp64": 1e-12, "mixed": 5e-6}




def system(grid, seed=3):
    s = synth.water_box(216, 18.63, 24, seed, "water_648")
    s.grid = tuple(grid)
    return s


GRIDS = [(24, 24, 24), (20, 21, 28), (30, 25, 18), (28, 15, 35), (10, 12, 14)]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plane_field_matches_oracle_and_bricks(grid, prec):
    print(f"[gpu] plane field grid={grid} {prec}", flush=True)
    s = system(grid)
    rng = np.random.default_rng(11)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    ref_rec = O.spme_field(s, dip=mu)
    ref_mv = O.matvec(s, mu, "spme")
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        assert ctx.info()["pme_planes"] == 1
        mu_d = torch.tensor(mu, device=DEV)
        _, ek = ctx.dipole_field_parts(t["pos"], mu_d)
        ek = ek.cpu().numpy()
        q = ctx.dipole_matvec(t["pos"], mu_d).cpu().numpy()
        ctx.set_pme_path("bricks")
        assert ctx.info()["pme_planes"] == 0
        _, ek_b = ctx.dipole_field_parts(t["pos"], mu_d)
        ek_b = ek_b.cpu().numpy()
        q_b = ctx.dipole_matvec(t["pos"], mu_d).cpu().numpy()
    finally:
        ctx.close()
    assert_fields(ek, ref_rec, TOL[prec], what="recip field vs oracle")
    assert_fields(q, ref_mv, 1e-12 if prec == "fp64" else 2e-6, what="matvec vs oracle")
    assert_fields(ek, ek_b, TOL_PATHS[prec], what="recip field planes vs bricks")
    assert_fields(q, q_b, TOL_PATHS[prec], what="matvec planes vs bricks")


@pytest.mark.parametrize("grid", [(24, 24, 24), (20, 21, 28), (28, 15, 35)], ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plane_perm_field_matches_oracle_and_bricks(grid, prec):
    """Permanent multipoles (charges, dipoles, quadrupoles) spread on the plane path."""
    print(f"[gpu] plane perm field grid={grid} {prec}", flush=True)
    s = system(grid)
    ref = O.perm_field(s, "spme")
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]).cpu().numpy()
        ctx.set_pme_path("bricks")
        e_b = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]).cpu().numpy()
    finally:
        ctx.close()
    assert_fields(e, ref, (1e-11 if prec == "fp64" else 2e-5))
    assert_fields(e, e_b, TOL_PATHS[prec])


def test_plane_mixed_is_bitwise_reproducible():
    s = system((20, 21, 28))
    rng = np.random.default_rng(5)
    mu = torch.tensor(rng.standard_normal((s.n, 3)) * 0.05, device=DEV)
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    try:
        a = ctx.dipole_field_parts(t["pos"], mu)[1].clone()
        # a different list build of the same configuration refills the x-bins in another order
        ctx.build_blocklist(t["pos"])
        b = ctx.dipole_field_parts(t["pos"], mu)[1].clone()
    finally:
        ctx.close()
    assert torch.equal(a, b)


def test_plane_solve_matches_oracle():
    s = system((20, 21, 28))
    e_ref = O.perm_field(s, "spme")
    mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-10)
    e_gpu = torch.tensor(e_ref, device=DEV)
    for prec in ("fp64", "mixed"):
        ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
        try:
            assert ctx.info()["pme_planes"] == 1
            mu, ep, it, st = ctx.polarize(t["pos"], e_gpu, tol_debye=1e-7, max_iter=200)
        finally:
            ctx.close()
        assert st == amoeba.AMOEBA_OK
        err = O.rms_debye(mu.cpu().numpy() - mu_ref)
        assert err < (2e-7 if prec == "fp64" else 1e-5), (prec, err)


def test_grid_outside_plane_path_falls_back_to_bricks():
    s = system((22, 24, 24))   # 22 = 2 x 11: no radix for 11
    rng = np.random.default_rng(2)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    ref = O.spme_field(s, dip=mu)
    ctx, t = amoeba.context_for(s, precision="fp64", device=DEV)
    try:
        assert ctx.info()["pme_planes"] == 0
        with pytest.raises(amoeba.AmoebaError):
            ctx.set_pme_path("planes")
        ctx.set_pme_path("auto")
        _, ek = ctx.dipole_field_parts(t["pos"], torch.tensor(mu, device=DEV))
    finally:
        ctx.close()
    assert_fields(ek.cpu().numpy(), ref, TOL["fp64"])
