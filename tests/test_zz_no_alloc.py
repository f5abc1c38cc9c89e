"""The learned-guess gradient entry point that allocates nothing (for callers that cannot call
hipMalloc): through the C ABI it must return bitwise the loss and gradient of the ordinary
entry point, on two calls in a row (the second on a smaller batch, so that the library's static
scratch still holds the first call's partials), and against the FP64 oracle's backpropagation
to the FP32 bar of the ordinary entry point's own test.  Sizes beyond the scratch are rejected
on the host."""
import numpy as np
import pytest
import torch

from oracle import guess as G
from paper_2011_01207_amd import amoeba, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def f32(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device=DEV)


def model_with_last_layer(seed):
    rng = np.random.default_rng(seed)
    m = synth.guess_init_model(seed=seed).astype(np.float64)
    m[G.NPARAM - 3 * 64 - 3:G.NPARAM] = rng.standard_normal(3 * 64 + 3) * 0.3
    m[G.NPARAM:G.NPARAM + G.NFEAT] = rng.standard_normal(G.NFEAT) * 0.2
    m[G.NPARAM + G.NFEAT:] = rng.uniform(0.5, 2.0, G.NFEAT)
    return m.astype(np.float32)


def test_noalloc_gradient_equals_the_allocating_entry_point():
    print("[gpu] no-allocation guess gradient", flush=True)
    rng = np.random.default_rng(90)
    rows = 9000
    x = f32(rng.standard_normal((rows, G.NFEAT)))
    b = f32(rng.standard_normal((rows, 3, 3)) * 0.1)
    y = f32(rng.standard_normal((rows, 3)) * 0.1)
    model = model_with_last_layer(91)
    s = synth.water648()
    ctx, _ = amoeba.context_for(s, precision="mixed", device=DEV)
    try:
        ctx.guess_set_model(model)
        grad = torch.empty(amoeba.GUESS_NPARAM, dtype=torch.float32, device=DEV)
        # the largest accepted batch (128 workgroups of the scratch), then a smaller index batch
        idx2 = torch.tensor(rng.integers(0, rows, 777).astype(np.int32), device=DEV)
        for args in ({"n_batch": amoeba.GUESS_NOALLOC_MAX_BATCH}, {"idx": idx2}):
            l_ref, g_ref = ctx.guess_gradient(x, b, y, **args)
            l_na, g_na = ctx.guess_gradient_noalloc(x, b, y, out=grad, **args)
            assert l_na == l_ref
            assert torch.equal(g_na, g_ref)
            sel = np.arange(amoeba.GUESS_NOALLOC_MAX_BATCH) if "n_batch" in args else idx2.cpu().numpy()
            l_o, g_o = G.loss_grad(model.astype(np.float64), x.cpu().numpy()[sel].astype(np.float64),
                                   b.cpu().numpy()[sel].astype(np.float64), y.cpu().numpy()[sel].astype(np.float64))
            assert abs(l_na - l_o) < 1e-5 * l_o
            g = g_na.cpu().numpy().astype(np.float64)
            assert np.linalg.norm(g - g_o) < 1e-4 * np.linalg.norm(g_o)
        # the delta kind's offsets reach the scratch path too
        ctx.guess_set_kind("delta")
        l_ref, g_ref = ctx.guess_gradient(x, b, y, n_batch=1000)
        l_na, g_na = ctx.guess_gradient_noalloc(x, b, y, n_batch=1000, out=grad)
        assert l_na == l_ref and torch.equal(g_na, g_ref)
        # beyond the scratch: rejected before any launch
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.guess_gradient_noalloc(x, b, y, n_batch=amoeba.GUESS_NOALLOC_MAX_BATCH + 1, out=grad)
        assert ei.value.status == amoeba.AMOEBA_E_INVALID
    finally:
        ctx.close()
