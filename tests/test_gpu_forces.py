"""GPU parity of the polarization energy gradient (amoeba_polarization_gradient) against the
FP64 oracle's analytic gradient, which the CPU tests pin to central differences of the oracle's
own E_pol.  The dipoles are the oracle's exact solution, so both sides differentiate the same
stationary energy; the comparison is atom by atom (rms and per-atom maximum)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2011_01207_amd import amoeba, synth
from parity_util import assert_fields

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"
BAR = {"fp64": 1e-10, "mixed": 3e-5}
CASES = {"water_648": synth.water648, "solvated_chain_23558": synth.solvated_chain}
_REF = {}


def reference(name):
    if name not in _REF:
        s = CASES[name]()
        print(f"[gpu] oracle gradient {name} (N={s.n})", flush=True)
        e = O.perm_field(s, "spme")
        mu, _, _ = O.pcg(s, e, "spme", tol_debye=1e-10)
        _REF[name] = (s, mu, O.polar_gradient(s, mu, "spme"))
    return _REF[name]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_gradient_matches_oracle(name, prec):
    s, mu, g_ref = reference(name)
    print(f"[gpu] polarization gradient {name} {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        g = ctx.polarization_gradient(t["pos"], t["q"], t["dip"], t["quad"], torch.tensor(mu, device=DEV))
        g = g.cpu().numpy()
        # the same call twice: mixed precision sums in fixed point (bitwise), FP64 to rounding
        g2 = ctx.polarization_gradient(t["pos"], t["q"], t["dip"], t["quad"], torch.tensor(mu, device=DEV))
        g2 = g2.cpu().numpy()
    finally:
        ctx.close()
    assert_fields(g, g_ref, BAR[prec], what=f"dE_pol/dr {name} {prec}")
    if prec == "mixed":
        assert np.array_equal(g, g2)
    else:
        assert np.max(np.abs(g - g2)) <= 1e-12 * np.max(np.abs(g))


def test_gradient_error_paths():
    s = synth.water648()
    ctx, t = amoeba.context_for(s, precision="fp64", device=DEV)
    try:
        mu = torch.zeros_like(t["pos"])
        qbad = t["quad"].clone()
        qbad[3, 0] += 1e-6
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.polarization_gradient(t["pos"], t["q"], t["dip"], qbad, mu)
        assert ei.value.status == amoeba.AMOEBA_E_INVALID
        mu[2, 1] = float("nan")
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.polarization_gradient(t["pos"], t["q"], t["dip"], t["quad"], mu)
        assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.polarization_gradient(t["pos"] + 0.01, t["q"], t["dip"], t["quad"], torch.zeros_like(mu))
        assert ei.value.status == amoeba.AMOEBA_E_LIST
    finally:
        ctx.close()
