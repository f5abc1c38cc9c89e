"""GPU tests of the stage timers: AMOEBA_TIMING_STAGES times every stage alone, AMOEBA_TIMING_LIVE
only the real-space tiles where they run (second stream); live timing leaves the results
bitwise as they are, the stage pass to rounding."""
import pytest
import torch

import oracle as O
from paper_2011_01207_amd import amoeba, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def test_timing_modes():
    print("[gpu] timing modes", flush=True)
    s = synth.water_box(216, 18.63, 24, 3, "water_648")
    e = torch.tensor(O.perm_field(s, "spme"), device=DEV)
    ctx, t = amoeba.context_for(s, precision="mixed", device=DEV)
    try:
        ref = ctx.polarize(t["pos"], e, tol_debye=1e-7, max_iter=200)[0].clone()
        res = {}
        for mode in ("live", "stages"):
            ctx.set_timing(mode)
            mu = ctx.polarize(t["pos"], e, tol_debye=1e-7, max_iter=200)[0].clone()
            res[mode] = (mu, ctx.timing())
        ctx.set_timing("off")
        with pytest.raises(amoeba.AmoebaError):
            ctx.set_timing(7)
    finally:
        ctx.close()
    mu_l, tl = res["live"]
    mu_s, ts = res["stages"]
    # live timing leaves the products as they are; the stage pass runs the real-space and
    # reciprocal parts one after the other, which may round the last bit of a sum differently
    assert torch.equal(mu_l, ref)
    assert float((mu_s - ref).abs().max()) < 1e-12 * float(ref.abs().max())
    assert tl["launches"]["real"] > 0 and tl["ms"]["real"] > 0
    assert all(tl["launches"][k] == 0 for k in tl["launches"] if k != "real")
    for k in ("real", "spread", "fft", "gather", "pcg"):
        assert ts["launches"][k] > 0 and ts["ms"][k] > 0, k
    assert tl["matvecs"] == ts["matvecs"] > 0
