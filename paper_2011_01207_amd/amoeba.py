"""ctypes binding of libamoeba.so (include/amoeba.h).

Argument marshalling only: tensors are checked for device, dtype, shape and contiguity and
their device pointers are handed to the C entry points of the same names; every step of the
computation runs in the library's HIP kernels.  There is no fallback: if the built library or
a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamoeba.so")

AMOEBA_OK = 0
AMOEBA_NOT_CONVERGED = 1
AMOEBA_E_INVALID = -1
AMOEBA_E_NOMEM = -2
AMOEBA_E_DEVICE = -3
AMOEBA_E_LIST = -4
AMOEBA_E_OVERFLOW = -5
AMOEBA_E_NUMERIC = -6
AMOEBA_E_STATE = -7
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_LIST",
                -5: "E_OVERFLOW", -6: "E_NUMERIC", -7: "E_STATE"}

AMOEBA_FP64 = 0
AMOEBA_MIXED = 1
AMOEBA_GUESS_ZERO = 0
AMOEBA_GUESS_GIVEN = 1
AMOEBA_GUESS_LEARNED = 2
AMOEBA_GUESS_BEST = 3
GUESS_NAMES = {0: "zero", 1: "given", 2: "learned", 3: "best"}
AMOEBA_PME_AUTO = 0
AMOEBA_PME_PLANES = 1
AMOEBA_PME_BRICKS = 2
PME_PATHS = {"auto": 0, "planes": 1, "bricks": 2}
PAIR_STORE = {"auto": 0, "compute": 1, "stored": 2}
TIMING_MODES = {"off": 0, "stages": 1, "live": 2}
STAGE_NAMES = ["list", "perm", "real", "spread", "fft", "gather", "pcg", "guess"]

GUESS_NFEAT = 11
GUESS_NBASIS = 3
GUESS_HIDDEN = 64
GUESS_NPARAM = 5123
GUESS_NMODEL = 5145
GUESS_KINDS = {"neumann": 0, "delta": 1}
GUESS_BLOB_VERSION = 1
GUESS_BLOB_BYTES = 48 + 4 * (GUESS_NMODEL + 2 * GUESS_NPARAM)
GUESS_NOALLOC_MAX_BATCH = 8192
N_STAGES = 8


class amoeba_params(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("box", ctypes.c_double * 3), ("cutoff", ctypes.c_double),
                ("buffer", ctypes.c_double), ("ewald_alpha", ctypes.c_double), ("grid", ctypes.c_int32 * 3),
                ("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_workspace_bytes", ctypes.c_int64)]


class amoeba_info(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_blocks", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("last_iterations", ctypes.c_int32), ("last_rms_debye", ctypes.c_double),
                ("last_guess", ctypes.c_int32), ("guess_loaded", ctypes.c_int32),
                ("last_guess_rms_debye", ctypes.c_double * 2), ("pair_min_image", ctypes.c_int32),
                ("pme_planes", ctypes.c_int32),
                ("pair_store", ctypes.c_int32),
                ("pair_store_bytes", ctypes.c_int64)]


class amoeba_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * N_STAGES), ("launches", ctypes.c_int64 * N_STAGES),
                ("matvecs", ctypes.c_int64)]


class AmoebaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load libamoeba.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2011_01207_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.amoeba_create.argtypes = [ctypes.POINTER(amoeba_params), _P, ctypes.POINTER(_P)]
        L.amoeba_destroy.argtypes = [_P]
        L.amoeba_last_error.argtypes = [_P]
        L.amoeba_last_error.restype = ctypes.c_char_p
        L.amoeba_create_error.argtypes = []
        L.amoeba_create_error.restype = ctypes.c_char_p
        L.amoeba_set_atoms.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.c_int64]
        L.amoeba_build_blocklist.argtypes = [_P, _P]
        L.amoeba_update_blocklist.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int32)]
        L.amoeba_perm_field.argtypes = [_P, _P, _P, _P, _P, _P]
        L.amoeba_set_direct_scales.argtypes = [_P, _P, ctypes.c_int64]
        L.amoeba_perm_field_dp.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.amoeba_polarize_dp.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
        L.amoeba_dipole_matvec.argtypes = [_P, _P, _P, _P]
        L.amoeba_dipole_field_parts.argtypes = [_P, _P, _P, _P, _P]
        L.amoeba_polarization_gradient.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.amoeba_polarize_configuration.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_double,
                                                    ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double),
                                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.amoeba_polarize.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
        L.amoeba_get_info.argtypes = [_P, ctypes.POINTER(amoeba_info)]
        _fp = ctypes.POINTER(ctypes.c_float)
        L.amoeba_guess_set_model.argtypes = [_P, _fp, ctypes.c_int64]
        L.amoeba_guess_get_model.argtypes = [_P, _fp, ctypes.c_int64]
        L.amoeba_guess_features.argtypes = [_P, _P, _P, _P, _P]
        L.amoeba_guess_fit_norm.argtypes = [_P, _P, ctypes.c_int64]
        L.amoeba_guess_forward.argtypes = [_P, _P, _P, ctypes.c_int64, _P]
        L.amoeba_guess_gradient.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P,
                                            ctypes.POINTER(ctypes.c_double)]
        L.amoeba_guess_train_step.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_float,
                                              ctypes.POINTER(ctypes.c_double)]
        L.amoeba_guess_predict.argtypes = [_P, _P, _P, _P]
        L.amoeba_guess_gradient_noalloc.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P,
                                                     ctypes.POINTER(ctypes.c_double)]
        L.amoeba_guess_set_kind.argtypes = [_P, ctypes.c_int32]
        L.amoeba_guess_set_reference.argtypes = [_P, _P, _P]
        L.amoeba_guess_save.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int64)]
        L.amoeba_guess_load.argtypes = [_P, _P, ctypes.c_int64]
        L.amoeba_set_pme_path.argtypes = [_P, ctypes.c_int32]
        L.amoeba_set_pair_store.argtypes = [_P, ctypes.c_int32]
        L.amoeba_set_residual_check.argtypes = [_P, ctypes.c_int32]
        L.amoeba_set_graphs.argtypes = [_P, ctypes.c_int32]
        L.amoeba_set_timing.argtypes = [_P, ctypes.c_int]
        L.amoeba_get_timing.argtypes = [_P, ctypes.POINTER(amoeba_timing)]
        _lib = L
    return _lib


def _ptr(t, dtype, shape=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


class Context:
    """One amoeba_ctx: a fixed system size, box and parameter set on the current device/stream."""

    def __init__(self, n_atoms, box, cutoff=7.0, buffer=0.0, ewald_alpha=0.545, grid=(24, 24, 24), order=5,
                 precision="fp64", max_workspace_bytes=0, stream=None):
        L = lib()
        p = amoeba_params()
        p.n_atoms = int(n_atoms)
        for a in range(3):
            p.box[a] = float(box[a])
            p.grid[a] = int(grid[a])
        p.cutoff, p.buffer, p.ewald_alpha = float(cutoff), float(buffer), float(ewald_alpha)
        p.order = int(order)
        p.precision = {"fp64": AMOEBA_FP64, "mixed": AMOEBA_MIXED}[precision] if isinstance(precision, str) \
            else int(precision)
        p.max_workspace_bytes = int(max_workspace_bytes)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
        self.stream = stream
        h = _P()
        st = L.amoeba_create(ctypes.byref(p), _P(stream), ctypes.byref(h))
        if st != AMOEBA_OK:
            raise AmoebaError(st, L.amoeba_create_error().decode())
        self.h = h
        self.n = int(n_atoms)
        self.params = p
        self.guess_kind = "neumann"    # mirrors the context's learned-guess kind

    def _check(self, st, ok=(AMOEBA_OK,)):
        if st not in ok:
            raise AmoebaError(st, lib().amoeba_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().amoeba_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # entry points ---------------------------------------------------------------------------
    def set_atoms(self, alpha, thole, sc_ptr, sc_j, sc_s):
        n = self.n
        nnz = int(sc_j.numel())
        return self._check(lib().amoeba_set_atoms(
            self.h, _ptr(alpha, torch.float64, (n,), "alpha"), _ptr(thole, torch.float64, (n,), "thole"),
            _ptr(sc_ptr, torch.int32, (n + 1,), "sc_ptr"),
            _ptr(sc_j, torch.int32, (nnz,), "sc_j") if nnz else None,
            _ptr(sc_s, torch.float64, (nnz,), "sc_s") if nnz else None, nnz))

    def set_direct_scales(self, sc_s_d):
        """Direct (d) scales of the pairs given to set_atoms, in the same order."""
        nnz = int(sc_s_d.numel())
        return self._check(lib().amoeba_set_direct_scales(
            self.h, _ptr(sc_s_d, torch.float64, (nnz,), "sc_s_d") if nnz else None, nnz))

    def build_blocklist(self, pos):
        return self._check(lib().amoeba_build_blocklist(self.h, _ptr(pos, torch.float64, (self.n, 3), "pos")))

    def update_blocklist(self, pos):
        """Rebuild the list only if none exists or an atom moved more than buffer/2 since the
        last build, else refresh the masks; returns True when it rebuilt."""
        r = ctypes.c_int32(0)
        self._check(lib().amoeba_update_blocklist(self.h, _ptr(pos, torch.float64, (self.n, 3), "pos"),
                                                  ctypes.byref(r)))
        return bool(r.value)

    def perm_field(self, pos, q, dip, quad, out=None):
        n = self.n
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        self._check(lib().amoeba_perm_field(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(q, torch.float64, (n,), "q"),
            _ptr(dip, torch.float64, (n, 3), "dip"), _ptr(quad, torch.float64, (n, 6), "quad"),
            _ptr(out, torch.float64, (n, 3), "e_perm")))
        return out

    def perm_field_dp(self, pos, q, dip, quad):
        """Returns (e_d, e_p): the permanent field with the direct and with the p-scales."""
        n = self.n
        e_d = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        e_p = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(lib().amoeba_perm_field_dp(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(q, torch.float64, (n,), "q"),
            _ptr(dip, torch.float64, (n, 3), "dip"), _ptr(quad, torch.float64, (n, 6), "quad"),
            _ptr(e_d, torch.float64, (n, 3), "e_d"), _ptr(e_p, torch.float64, (n, 3), "e_p")))
        return e_d, e_p

    def polarize_dp(self, pos, e_d, e_p, tol_debye=1e-5, max_iter=500):
        """Returns (mu_d, mu_p, e_pol kcal/mol, (iterations d, p), status)."""
        n = self.n
        mu_d = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        mu_p = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        ep = ctypes.c_double(0.0)
        its = (ctypes.c_int32 * 2)(0, 0)
        st = self._check(lib().amoeba_polarize_dp(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(e_d, torch.float64, (n, 3), "e_d"),
            _ptr(e_p, torch.float64, (n, 3), "e_p"), float(tol_debye), int(max_iter),
            _ptr(mu_d, torch.float64, (n, 3), "mu_d_out"), _ptr(mu_p, torch.float64, (n, 3), "mu_p_out"),
            ctypes.byref(ep), ctypes.cast(its, ctypes.POINTER(ctypes.c_int32))),
            ok=(AMOEBA_OK, AMOEBA_NOT_CONVERGED))
        return mu_d, mu_p, ep.value, (its[0], its[1]), st

    def dipole_matvec(self, pos, mu, out=None):
        n = self.n
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        self._check(lib().amoeba_dipole_matvec(self.h, _ptr(pos, torch.float64, (n, 3), "pos"),
                                               _ptr(mu, torch.float64, (n, 3), "mu"),
                                               _ptr(out, torch.float64, (n, 3), "out")))
        return out

    def dipole_field_parts(self, pos, mu):
        n = self.n
        er = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        ek = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(lib().amoeba_dipole_field_parts(self.h, _ptr(pos, torch.float64, (n, 3), "pos"),
                                                    _ptr(mu, torch.float64, (n, 3), "mu"), er.data_ptr(),
                                                    ek.data_ptr()))
        return er, ek

    def polarize(self, pos, e_perm, mu_guess=None, guess_mode=None, tol_debye=1e-5, max_iter=500, out=None):
        """Returns (mu, e_pol kcal/mol, iterations, status); status is OK or NOT_CONVERGED.
        guess_mode: None (zero, or given when mu_guess is passed), an AMOEBA_GUESS_* value or one
        of "zero", "given", "learned", "best"."""
        n = self.n
        if isinstance(guess_mode, str):
            guess_mode = {v: k for k, v in GUESS_NAMES.items()}[guess_mode]
        if guess_mode is None:
            guess_mode = AMOEBA_GUESS_ZERO if mu_guess is None else AMOEBA_GUESS_GIVEN
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        ep = ctypes.c_double(0.0)
        it = ctypes.c_int32(0)
        st = self._check(lib().amoeba_polarize(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(e_perm, torch.float64, (n, 3), "e_perm"),
            _ptr(mu_guess, torch.float64, (n, 3), "mu_guess"), int(guess_mode), float(tol_debye), int(max_iter),
            _ptr(out, torch.float64, (n, 3), "mu_out"), ctypes.byref(ep), ctypes.byref(it)),
            ok=(AMOEBA_OK, AMOEBA_NOT_CONVERGED))
        return out, ep.value, it.value, st

    def polarize_configuration(self, pos, q, dip, quad, mu_guess=None, guess_mode=None, tol_debye=1e-5,
                               max_iter=500, out=None, e_perm_out=None):
        """update_blocklist + perm_field + polarize in one call.  Returns (mu, e_perm, e_pol
        kcal/mol, iterations, status, rebuilt); e_perm is None unless e_perm_out is given."""
        n = self.n
        if isinstance(guess_mode, str):
            guess_mode = {v: k for k, v in GUESS_NAMES.items()}[guess_mode]
        if guess_mode is None:
            guess_mode = AMOEBA_GUESS_ZERO if mu_guess is None else AMOEBA_GUESS_GIVEN
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        ep = ctypes.c_double(0.0)
        it = ctypes.c_int32(0)
        rb = ctypes.c_int32(0)
        st = self._check(lib().amoeba_polarize_configuration(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(q, torch.float64, (n,), "q"),
            _ptr(dip, torch.float64, (n, 3), "dip"), _ptr(quad, torch.float64, (n, 6), "quad"),
            _ptr(mu_guess, torch.float64, (n, 3), "mu_guess"), int(guess_mode), float(tol_debye), int(max_iter),
            _ptr(e_perm_out, torch.float64, (n, 3), "e_perm_out"), _ptr(out, torch.float64, (n, 3), "mu_out"),
            ctypes.byref(ep), ctypes.byref(it), ctypes.byref(rb)),
            ok=(AMOEBA_OK, AMOEBA_NOT_CONVERGED))
        return out, e_perm_out, ep.value, it.value, st, bool(rb.value)

    def polarization_gradient(self, pos, q, dip, quad, mu, out=None):
        """dE_pol/dr (kcal/mol/A, N x 3 on the device) at the induced dipoles mu."""
        n = self.n
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        self._check(lib().amoeba_polarization_gradient(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(q, torch.float64, (n,), "q"),
            _ptr(dip, torch.float64, (n, 3), "dip"), _ptr(quad, torch.float64, (n, 6), "quad"),
            _ptr(mu, torch.float64, (n, 3), "mu"), _ptr(out, torch.float64, (n, 3), "grad_out")))
        return out

    def set_pme_path(self, path):
        """path: "auto", "planes" or "bricks" (or the AMOEBA_PME_* value)."""
        self._check(lib().amoeba_set_pme_path(self.h, PME_PATHS[path] if isinstance(path, str) else int(path)))

    def set_pair_store(self, mode):
        """mode: "auto", "compute" or "stored" (or the AMOEBA_PAIRS_* value)."""
        self._check(lib().amoeba_set_pair_store(self.h, PAIR_STORE[mode] if isinstance(mode, str) else int(mode)))

    def set_timing(self, mode):
        """mode: "off", "stages" or "live" (or the AMOEBA_TIMING_* value); resets the counters."""
        self._check(lib().amoeba_set_timing(self.h, TIMING_MODES[mode] if isinstance(mode, str) else int(mode)))

    def timing(self) -> dict:
        """Milliseconds and launches per stage since set_timing, and the working products."""
        t = amoeba_timing()
        self._check(lib().amoeba_get_timing(self.h, ctypes.byref(t)))
        return {"ms": {STAGE_NAMES[i]: t.ms[i] for i in range(N_STAGES)},
                "launches": {STAGE_NAMES[i]: int(t.launches[i]) for i in range(N_STAGES)},
                "matvecs": int(t.matvecs)}

    def set_residual_check(self, mode):
        """mode: "auto" (the default) or "always"."""
        m = {"auto": 0, "always": 1}[mode] if isinstance(mode, str) else int(mode)
        return self._check(lib().amoeba_set_residual_check(self.h, m))

    def set_graphs(self, enable):
        """Run PCG iterations as one captured HIP graph each (True) or as individual kernel
        launches (False, the library's default)."""
        self._check(lib().amoeba_set_graphs(self.h, 1 if enable else 0))

    def info(self) -> dict:
        inf = amoeba_info()
        self._check(lib().amoeba_get_info(self.h, ctypes.byref(inf)))
        out = {k: getattr(inf, k) for k, _ in amoeba_info._fields_}
        out["last_guess_rms_debye"] = tuple(out["last_guess_rms_debye"])
        return out

    # learned initial guess ------------------------------------------------------------------
    def guess_set_model(self, model):
        """model: host float32 array-like of GUESS_NMODEL entries."""
        import numpy as np
        m = np.ascontiguousarray(np.asarray(model, dtype=np.float32).ravel())
        return self._check(lib().amoeba_guess_set_model(
            self.h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), m.size))

    def guess_get_model(self):
        import numpy as np
        m = np.empty(GUESS_NMODEL, dtype=np.float32)
        self._check(lib().amoeba_guess_get_model(self.h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), m.size))
        return m

    def guess_set_kind(self, kind):
        """'neumann' (bases from two real-space products) or 'delta' (previous-configuration
        reference, no product)."""
        self._check(lib().amoeba_guess_set_kind(self.h, GUESS_KINDS[kind]))
        self.guess_kind = kind

    def guess_set_reference(self, mu_ref, e_ref):
        """Converged dipoles and permanent field of the previous configuration (device FP64,
        caller order), copied into the context for the delta kind."""
        n = self.n
        return self._check(lib().amoeba_guess_set_reference(
            self.h, _ptr(mu_ref, torch.float64, (n, 3), "mu_ref"), _ptr(e_ref, torch.float64, (n, 3), "e_ref")))

    def guess_save(self) -> bytes:
        """Versioned checkpoint (kind, model, Adam moments and step count) as bytes."""
        size = ctypes.c_int64(0)
        self._check(lib().amoeba_guess_save(self.h, None, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        self._check(lib().amoeba_guess_save(self.h, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(size)))
        return buf.raw[:size.value]

    def guess_load(self, blob: bytes):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(lib().amoeba_guess_load(self.h, ctypes.cast(buf, ctypes.c_void_p), len(blob)))
        kind = int.from_bytes(bytes(blob)[12:16], "little", signed=True)
        self.guess_kind = {v: k for k, v in GUESS_KINDS.items()}[kind]

    def guess_features(self, pos, e_perm, feat=None, basis=None):
        """(feat [N][NFEAT], basis [N][NBASIS][3]) FP32 on the device, caller order."""
        n = self.n
        feat = torch.empty((n, GUESS_NFEAT), dtype=torch.float32, device=pos.device) if feat is None else feat
        basis = torch.empty((n, GUESS_NBASIS, 3), dtype=torch.float32, device=pos.device) if basis is None else basis
        self._check(lib().amoeba_guess_features(
            self.h, _ptr(pos, torch.float64, (n, 3), "pos"), _ptr(e_perm, torch.float64, (n, 3), "e_perm"),
            _ptr(feat, torch.float32, (n, GUESS_NFEAT), "feat"),
            _ptr(basis, torch.float32, (n, GUESS_NBASIS, 3), "basis")))
        return feat, basis

    def guess_fit_norm(self, feat):
        rows = int(feat.shape[0])
        return self._check(lib().amoeba_guess_fit_norm(
            self.h, _ptr(feat, torch.float32, (rows, GUESS_NFEAT), "feat"), rows))

    def guess_forward(self, feat, basis, out=None):
        rows = int(feat.shape[0])
        out = torch.empty((rows, 3), dtype=torch.float32, device=feat.device) if out is None else out
        self._check(lib().amoeba_guess_forward(
            self.h, _ptr(feat, torch.float32, (rows, GUESS_NFEAT), "feat"),
            _ptr(basis, torch.float32, (rows, GUESS_NBASIS, 3), "basis"), rows,
            _ptr(out, torch.float32, (rows, 3), "mu_out")))
        return out

    def _batch_args(self, feat, basis, target, idx, n_batch):
        rows = int(feat.shape[0])
        if idx is not None:
            n_batch = int(idx.numel())
            ip = _ptr(idx, torch.int32, (n_batch,), "idx")
        else:
            n_batch = rows if n_batch is None else int(n_batch)
            ip = None
        return (_ptr(feat, torch.float32, (rows, GUESS_NFEAT), "feat"),
                _ptr(basis, torch.float32, (rows, GUESS_NBASIS, 3), "basis"),
                _ptr(target, torch.float32, (rows, 3), "target"), rows, ip, n_batch)

    def guess_gradient(self, feat, basis, target, idx=None, n_batch=None):
        """(loss in D^2, gradient [NPARAM] FP32 on the device) of a batch; the model is unchanged."""
        g = torch.empty(GUESS_NPARAM, dtype=torch.float32, device=feat.device)
        loss = ctypes.c_double(0.0)
        self._check(lib().amoeba_guess_gradient(self.h, *self._batch_args(feat, basis, target, idx, n_batch),
                                                g.data_ptr(), ctypes.byref(loss)))
        return loss.value, g

    def guess_gradient_noalloc(self, feat, basis, target, idx=None, n_batch=None, out=None):
        """guess_gradient through the entry point that allocates nothing (library scratch); the
        caller passes the gradient tensor (FP32 [NPARAM] on the device) to stay allocation-free."""
        g = torch.empty(GUESS_NPARAM, dtype=torch.float32, device=feat.device) if out is None else out
        loss = ctypes.c_double(0.0)
        self._check(lib().amoeba_guess_gradient_noalloc(
            self.h, *self._batch_args(feat, basis, target, idx, n_batch),
            _ptr(g, torch.float32, (GUESS_NPARAM,), "grad_out"), ctypes.byref(loss)))
        return loss.value, g

    def guess_train_step(self, feat, basis, target, lr, idx=None, n_batch=None):
        """One Adam step; returns the batch loss (D^2) before the step."""
        loss = ctypes.c_double(0.0)
        self._check(lib().amoeba_guess_train_step(self.h, *self._batch_args(feat, basis, target, idx, n_batch),
                                                  float(lr), ctypes.byref(loss)))
        return loss.value

    def guess_predict(self, pos, e_perm, out=None):
        n = self.n
        out = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if out is None else out
        self._check(lib().amoeba_guess_predict(self.h, _ptr(pos, torch.float64, (n, 3), "pos"),
                                               _ptr(e_perm, torch.float64, (n, 3), "e_perm"),
                                               _ptr(out, torch.float64, (n, 3), "mu0_out")))
        return out


def context_for(system, precision="fp64", device="cuda", **kw):
    """Create a Context for a synthetic System and upload its parameters; returns
    (ctx, tensors dict) with pos, q, dip, quad, alpha, thole and the scaled-pair CSR on device."""
    t = {
        "pos": torch.tensor(system.pos, dtype=torch.float64, device=device),
        "q": torch.tensor(system.q, dtype=torch.float64, device=device),
        "dip": torch.tensor(system.dip, dtype=torch.float64, device=device),
        "quad": torch.tensor(system.quad, dtype=torch.float64, device=device),
        "alpha": torch.tensor(system.alpha, dtype=torch.float64, device=device),
        "thole": torch.tensor(system.thole, dtype=torch.float64, device=device),
        "sc_ptr": torch.tensor(system.sc_ptr, dtype=torch.int32, device=device),
        "sc_j": torch.tensor(system.sc_j, dtype=torch.int32, device=device),
        "sc_s": torch.tensor(system.sc_s, dtype=torch.float64, device=device),
    }
    ctx = Context(system.n, system.box, cutoff=system.cutoff, buffer=system.buffer,
                  ewald_alpha=system.ewald_alpha, grid=system.grid, order=system.order, precision=precision, **kw)
    ctx.set_atoms(t["alpha"], t["thole"], t["sc_ptr"], t["sc_j"], t["sc_s"])
    if getattr(system, "sc_s_d", None) is not None:
        t["sc_s_d"] = torch.tensor(system.sc_s_d, dtype=torch.float64, device=device)
        ctx.set_direct_scales(t["sc_s_d"])
    ctx.build_blocklist(t["pos"])
    return ctx, t
