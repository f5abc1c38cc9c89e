"""Element-wise parity checks shared by the GPU tests.

A field (or any per-atom vector quantity, N x 3) is compared atom by atom: the rms of the
per-atom error and its maximum, both relative to the rms magnitude of the reference.  The rms
bound is the test's bar; the maximum is held to a stated multiple of it, so that a single wrong
atom or one bad tile (an error of the order of the field itself) cannot hide inside the rms,
while the spread of ordinary rounding over many atoms (a few times the rms) passes."""
import numpy as np

MAX_FACTOR = 50.0   # per-atom maximum allowed, as a multiple of the rms bar


def field_errors(a, b):
    """(rms, max) over atoms of |a_i - b_i|, both divided by the rms of |b_i|."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    scale = float(np.sqrt(np.mean(np.sum(b * b, axis=1))))
    d = np.linalg.norm(a - b, axis=1)
    return float(np.sqrt(np.mean(d * d))) / scale, float(np.max(d)) / scale


def rel_rms(a, b):
    return field_errors(a, b)[0]


def assert_fields(a, b, bar, max_factor=MAX_FACTOR, what="field"):
    r, m = field_errors(a, b)
    print(f"  {what}: rel rms {r:.3e} (bar {bar:.1e}), rel max {m:.3e} (bar {max_factor * bar:.1e})", flush=True)
    assert r < bar, f"{what}: relative rms error {r:.3e} >= {bar:.1e}"
    assert m < max_factor * bar, f"{what}: relative per-atom max error {m:.3e} >= {max_factor * bar:.1e}"
