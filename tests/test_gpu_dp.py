"""GPU parity of the two-set (direct / polarization) model against the FP64 oracle.

The direct scales change only the permanent field the d set is driven by; both sets are solved
with the same operator.  Checked here: both permanent fields, both converged dipole sets and the
two-set energy against the oracle, the p set against the one-set solve of the same field, and
the entry points' error paths."""
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
def sys_dp():
    return synth.solvated_chain_small()


@pytest.fixture(scope="module")
def ref_dp(sys_dp):
    e_d, e_p = O.perm_field_dp(sys_dp, "spme")
    mu_d, _, _ = O.pcg(sys_dp, e_d, "spme", tol_debye=1e-10)
    mu_p, _, _ = O.pcg(sys_dp, e_p, "spme", tol_debye=1e-10)
    return {"e_d": e_d, "e_p": e_p, "mu_d": mu_d, "mu_p": mu_p, "e_pol": O.e_pol_dp(mu_d, e_p)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dp_fields_and_solve(sys_dp, ref_dp, prec):
    print(f"[gpu] d/p two-set {prec}, {sys_dp.n} atoms", flush=True)
    ctx, t = amoeba.context_for(sys_dp, precision=prec, device=DEV)
    e_d, e_p = ctx.perm_field_dp(t["pos"], t["q"], t["dip"], t["quad"])
    tol = 1e-11 if prec == "fp64" else 3e-5
    assert_fields(e_d.cpu().numpy(), ref_dp["e_d"], tol, what="E_d")
    assert_fields(e_p.cpu().numpy(), ref_dp["e_p"], tol, what="E_p")
    # the p field is the one-set permanent field (bit for bit with the deterministic fixed-point
    # sums of the mixed mode; FP64 atomics add in any order)
    e1 = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    if prec == "mixed":
        assert torch.equal(e1, e_p)
    else:
        assert_fields(e1.cpu().numpy(), e_p.cpu().numpy(), 1e-14, what="E_perm vs E_p")
    # the fields differ where the scales do
    assert O.rms_debye((e_d - e_p).cpu().numpy()) > 0
    tol_s = 1e-8 if prec == "fp64" else 1e-6
    mu_d, mu_p, ep, its, st = ctx.polarize_dp(t["pos"], e_d, e_p, tol_debye=tol_s)
    assert st == amoeba.AMOEBA_OK and min(its) > 0
    bar = 1e-7 if prec == "fp64" else 1e-5
    assert O.rms_debye(mu_d.cpu().numpy() - ref_dp["mu_d"]) < bar
    assert O.rms_debye(mu_p.cpu().numpy() - ref_dp["mu_p"]) < bar
    assert O.rms_debye(ref_dp["mu_d"] - ref_dp["mu_p"]) > 100 * bar   # the sets really differ
    assert abs(ep - ref_dp["e_pol"]) < (1e-8 if prec == "fp64" else 1e-5) * abs(ref_dp["e_pol"])
    # E_pol is -1/2 C mu_d . e_p of the returned arrays
    assert abs(ep - O.e_pol_dp(mu_d.cpu().numpy(), e_p.cpu().numpy())) < 1e-10 * abs(ep)
    # the p set is the one-set solve of the same field from zero (bit for bit in mixed mode)
    m1, _, it1, st1 = ctx.polarize(t["pos"], e_p, tol_debye=tol_s)
    assert st1 == amoeba.AMOEBA_OK
    if prec == "mixed":
        assert torch.equal(m1, mu_p) and it1 == its[1]
    else:
        assert O.rms_debye((m1 - mu_p).cpu().numpy()) < 1e-9 and abs(it1 - its[1]) <= 1
    ctx.close()


def test_dp_without_direct_scales_gives_one_set(sys_dp):
    import dataclasses
    s = dataclasses.replace(sys_dp, sc_s_d=None)
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    e_d, e_p = ctx.perm_field_dp(t["pos"], t["q"], t["dip"], t["quad"])
    assert torch.equal(e_d, e_p)
    mu_d, mu_p, ep, its, st = ctx.polarize_dp(t["pos"], e_d, e_p, tol_debye=1e-6)
    assert st == amoeba.AMOEBA_OK and torch.equal(mu_d, mu_p) and its[0] == its[1]
    mu, ep1, _, _ = ctx.polarize(t["pos"], e_p, tol_debye=1e-6)
    assert torch.equal(mu, mu_p) and abs(ep - ep1) <= 1e-12 * abs(ep1)
    ctx.close()


def test_direct_scales_set_after_the_list_and_dropped_by_set_atoms(sys_dp):
    """Setting the direct scales after the list build takes effect on the next call; a new
    set_atoms drops them (both fields equal again)."""
    import dataclasses
    s = dataclasses.replace(sys_dp, sc_s_d=None)
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    ctx.set_direct_scales(torch.tensor(sys_dp.sc_s_d, device=DEV))
    e_d, e_p = ctx.perm_field_dp(t["pos"], t["q"], t["dip"], t["quad"])
    idx = np.arange(0, 60)
    e_d_ref, _ = O.perm_field_dp(sys_dp, "spme", idx=idx)
    assert_fields(e_d.cpu().numpy()[idx], e_d_ref, 3e-5, what="E_d (late scales)")
    ctx.set_atoms(t["alpha"], t["thole"], t["sc_ptr"], t["sc_j"], t["sc_s"])
    e_d2, e_p2 = ctx.perm_field_dp(t["pos"], t["q"], t["dip"], t["quad"])
    assert torch.equal(e_d2, e_p2) and torch.equal(e_p2, e_p)
    ctx.close()


def test_direct_scales_errors(sys_dp):
    ctx = amoeba.Context(sys_dp.n, sys_dp.box, cutoff=sys_dp.cutoff, ewald_alpha=sys_dp.ewald_alpha,
                         grid=sys_dp.grid, precision="fp64")
    sd = torch.tensor(sys_dp.sc_s_d, device=DEV)
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.set_direct_scales(sd)                      # before set_atoms
    assert e.value.status == amoeba.AMOEBA_E_STATE
    ctx.close()
    ctx, t = amoeba.context_for(sys_dp, precision="fp64", device=DEV)
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.set_direct_scales(sd[:-1])                 # wrong count
    assert e.value.status == amoeba.AMOEBA_E_INVALID
    bad = sd.clone()
    k = int(np.nonzero(sys_dp.sc_s_d != sys_dp.sc_s)[0][0])
    bad[k] = 0.25                                      # breaks the pair's symmetry
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.set_direct_scales(bad)
    assert e.value.status == amoeba.AMOEBA_E_INVALID
    bad = sd.clone()
    bad[k] = float("nan")
    with pytest.raises(amoeba.AmoebaError) as e:
        ctx.set_direct_scales(bad)
    assert e.value.status == amoeba.AMOEBA_E_INVALID
    # the context still works with its earlier scales
    e_d, e_p = ctx.perm_field_dp(t["pos"], t["q"], t["dip"], t["quad"])
    assert not torch.equal(e_d, e_p)
    ctx.close()
