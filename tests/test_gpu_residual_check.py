"""The true-residual check of mixed-precision solves: recomputed when the recursion may have
drifted (a start far from the solution), skipped when the drift bound is below a tenth of the
tolerance, with bitwise the same dipoles either way; every product is range-checked."""
import numpy as np
import pytest
import torch

from paper_2011_01207_amd import amoeba, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def products(ctx, pos, e, **kw):
    ctx.set_timing("live")   # resets the counters; leaves the products as they are
    mu, ep, it, st = ctx.polarize(pos, e, **kw)
    m = ctx.timing()["matvecs"]
    ctx.set_timing("off")
    assert st == amoeba.AMOEBA_OK
    return mu, ep, it, m


def test_check_is_skipped_only_where_it_cannot_matter():
    s = synth.water648()
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    try:
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        ref, _, _, _ = ctx.polarize(t["pos"], e, tol_debye=1e-9, max_iter=200)
        # zero start: sum of rms(z) ~ 0.1 D, the bound 2e-5 x that exceeds tol / 10: checked
        _, _, it0, m0 = products(ctx, t["pos"], e, tol_debye=1e-6)
        assert m0 == it0 + 1
        # a start 1e-4 e*A off the solution: the bound is far below tol / 10: not checked
        rng = np.random.default_rng(3)
        guess = ref + torch.tensor(rng.standard_normal((s.n, 3)) * 1e-4, device=DEV)
        mu_a, ep_a, it_a, m_a = products(ctx, t["pos"], e, mu_guess=guess, tol_debye=1e-6)
        assert m_a == it_a + 1           # the start's product and the iterations
        ctx.set_residual_check("always")
        mu_b, ep_b, it_b, m_b = products(ctx, t["pos"], e, mu_guess=guess, tol_debye=1e-6)
        assert m_b == it_b + 2           # and the check
        assert torch.equal(mu_a, mu_b) and ep_a == ep_b and it_a == it_b
        ctx.set_residual_check("auto")
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.set_residual_check(5)
        assert ei.value.status == amoeba.AMOEBA_E_INVALID
        # a start whose product leaves the exact fixed-point range: caught by the range check
        # of the start's product, with or without the final check
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.polarize(t["pos"], e * 1e5, mu_guess=ref * 1e5, tol_debye=1.0, max_iter=50)
        assert ei.value.status == amoeba.AMOEBA_E_OVERFLOW
        mu, _, _, st = ctx.polarize(t["pos"], e, tol_debye=1e-6)
        assert st == amoeba.AMOEBA_OK and torch.isfinite(mu).all()
    finally:
        ctx.close()
