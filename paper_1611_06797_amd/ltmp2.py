"""Thin ctypes binding of libltmp2 (argument marshalling only).

Every step of the LTMP2 path runs inside the HIP library; this module only
converts numpy arrays / torch device tensors into pointers and status codes
into exceptions.  PyTorch is used for device buffers and the current HIP
stream.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libltmp2.so")

STATUS = {0: "LTMP2_OK", 1: "LTMP2_EINVAL", 2: "LTMP2_EGAP", 3: "LTMP2_ENOMEM",
          4: "LTMP2_EDEVICE", 5: "LTMP2_ESTATE", 6: "LTMP2_ENUMERIC"}
FP64, FP32, BF16X3 = 0, 1, 2
QUAD_PLAIN, QUAD_LEARNED, QUAD_GIVEN = 0, 1, 2

EXPORTED = ("ltmp2_setup", "ltmp2_green", "ltmp2_chi", "ltmp2_exchange", "ltmp2_energy",
            "ltmp2_get_quadrature", "ltmp2_get_info", "ltmp2_aux_miller", "ltmp2_quadrature",
            "ltmp2_destroy", "ltmp2_last_error", "ltmp2_supported_grids", "ltmp2_set_timing",
            "ltmp2_get_timing", "ltmp2_mlp_init", "ltmp2_quadrature_table", "ltmp2_mlp_dataset",
            "ltmp2_mlp_forward", "ltmp2_mlp_grad", "ltmp2_mlp_train", "ltmp2_learned_quadrature",
            "ltmp2_mlp_last_error", "ltmp2_remez_polish", "ltmp2_batch_create",
            "ltmp2_batch_energy", "ltmp2_batch_info", "ltmp2_batch_group", "ltmp2_batch_cell",
            "ltmp2_batch_destroy", "ltmp2_batch_last_error", "ltmp2_batch_set_timing",
            "ltmp2_batch_get_timing", "ltmp2_real_orbitals", "ltmp2_mlp_forward_noalloc",
            "ltmp2_get_extrapolation", "ltmp2_direct_hartree", "ltmp2_setup_unrestricted",
            "ltmp2_setup_kpoints")
MLP_NPARAM = 5976
STAGES = ("chi_tiles", "chi_rows", "chi_cols", "w_gemm", "w_synth", "pair", "reduce")


class Params(C.Structure):
    _fields_ = [("L", C.c_double), ("n_fft", C.c_int), ("ecut", C.c_double),
                ("eaux", C.c_double), ("n_pw", C.c_int), ("n_states", C.c_int),
                ("n_occ", C.c_int),
                ("n_tau", C.c_int), ("quad_mode", C.c_int), ("prec", C.c_int),
                ("workspace_cap", C.c_size_t), ("n_extrap", C.c_int),
                ("extrap_alpha", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_r", C.c_int), ("n_g", C.c_int), ("n_h", C.c_int), ("n_pw", C.c_int),
                ("n_occ", C.c_int), ("n_vir", C.c_int), ("n_tau", C.c_int),
                ("x_min", C.c_double), ("x_max", C.c_double), ("quad_delta", C.c_double),
                ("device_bytes", C.c_size_t), ("quad_flags", C.c_int), ("n_grid", C.c_int),
                ("g_block", C.c_int), ("n_spin", C.c_int), ("n_occ_b", C.c_int),
                ("n_k", C.c_int)]


class BatchStats(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("n_groups", C.c_int), ("graph_ready", C.c_int),
                ("device_bytes", C.c_size_t)]


class LTMP2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libltmp2.so (import torch first so one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (shares its HIP runtime with the library)
    except ImportError:
        pass
    lib = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    lib.ltmp2_setup.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_char_p, C.c_void_p,
                                C.POINTER(C.c_void_p)]
    lib.ltmp2_setup_unrestricted.argtypes = [C.POINTER(Params), C.c_int] + [C.c_void_p] * 7 + [
        C.c_char_p, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.ltmp2_setup_kpoints.argtypes = [C.POINTER(Params), C.c_int] + [C.c_void_p] * 6 + [
        C.c_char_p, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.ltmp2_green.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    lib.ltmp2_chi.argtypes = [C.c_void_p, C.c_int, C.c_void_p, dp]
    lib.ltmp2_exchange.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp]
    lib.ltmp2_energy.argtypes = [C.c_void_p, dp, dp, C.c_void_p, dp]
    lib.ltmp2_get_quadrature.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, dp]
    lib.ltmp2_get_info.argtypes = [C.c_void_p, C.POINTER(Info)]
    lib.ltmp2_aux_miller.argtypes = [C.c_void_p, C.c_void_p]
    lib.ltmp2_quadrature.argtypes = [C.c_double, C.c_double, C.c_int, C.c_void_p, C.c_void_p, dp]
    lib.ltmp2_destroy.argtypes = [C.c_void_p]
    lib.ltmp2_destroy.restype = None
    lib.ltmp2_last_error.argtypes = [C.c_void_p]
    lib.ltmp2_last_error.restype = C.c_char_p
    lib.ltmp2_supported_grids.argtypes = [C.c_void_p, C.c_int]
    lib.ltmp2_set_timing.argtypes = [C.c_void_p, C.c_int]
    lib.ltmp2_get_timing.argtypes = [C.c_void_p, C.c_int, dp, C.POINTER(C.c_long)]
    vp = C.c_void_p
    lib.ltmp2_mlp_init.argtypes = [C.c_uint64, vp]
    lib.ltmp2_quadrature_table.argtypes = [C.c_int, C.c_int, vp, vp, vp, vp]
    lib.ltmp2_mlp_dataset.argtypes = [C.c_int, C.c_uint64, C.c_double, C.c_double, C.c_double,
                                      C.c_double, vp, C.c_int, vp, vp, vp, vp]
    lib.ltmp2_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
    lib.ltmp2_mlp_grad.argtypes = [vp, vp, vp, vp, C.c_int, vp, C.POINTER(C.c_float), vp]
    lib.ltmp2_mlp_train.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float,
                                    C.c_uint64, vp, vp]
    lib.ltmp2_learned_quadrature.argtypes = [vp, C.c_double, C.c_double, C.c_int, C.c_int,
                                             C.c_double, vp, vp, dp, C.POINTER(C.c_int), vp]
    lib.ltmp2_remez_polish.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, vp,
                                       vp, dp, C.POINTER(C.c_int)]
    lib.ltmp2_remez_polish.restype = C.c_int
    lib.ltmp2_batch_create.argtypes = [C.c_int, vp, vp, vp, vp, vp, vp, C.c_char_p, vp,
                                       C.POINTER(C.c_void_p)]
    lib.ltmp2_batch_energy.argtypes = [vp, vp, vp]
    lib.ltmp2_batch_info.argtypes = [vp, C.POINTER(BatchStats)]
    lib.ltmp2_batch_group.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      dp]
    lib.ltmp2_batch_cell.argtypes = [vp, C.c_int, C.POINTER(Info)]
    lib.ltmp2_batch_set_timing.argtypes = [vp, C.c_int]
    lib.ltmp2_batch_get_timing.argtypes = [vp, C.c_int, dp, C.POINTER(C.c_long)]
    lib.ltmp2_batch_destroy.argtypes = [vp]
    lib.ltmp2_batch_destroy.restype = None
    lib.ltmp2_batch_last_error.argtypes = [vp]
    lib.ltmp2_batch_last_error.restype = C.c_char_p
    lib.ltmp2_real_orbitals.argtypes = [C.c_int, vp, C.c_int, vp, C.c_int, vp, vp]
    lib.ltmp2_mlp_forward_noalloc.argtypes = [vp, vp, C.c_int, vp, vp]
    lib.ltmp2_get_extrapolation.argtypes = [vp, vp, vp, vp, vp]
    lib.ltmp2_direct_hartree.argtypes = [vp, C.c_int, dp]
    lib.ltmp2_mlp_last_error.argtypes = []
    lib.ltmp2_mlp_last_error.restype = C.c_char_p
    for name in ("ltmp2_setup", "ltmp2_green", "ltmp2_chi", "ltmp2_exchange", "ltmp2_energy",
                 "ltmp2_get_quadrature", "ltmp2_get_info", "ltmp2_aux_miller",
                 "ltmp2_quadrature", "ltmp2_set_timing", "ltmp2_get_timing", "ltmp2_mlp_init",
                 "ltmp2_quadrature_table", "ltmp2_mlp_dataset", "ltmp2_mlp_forward",
                 "ltmp2_mlp_grad", "ltmp2_mlp_train", "ltmp2_learned_quadrature",
                 "ltmp2_batch_create", "ltmp2_batch_energy", "ltmp2_batch_info",
                 "ltmp2_batch_group", "ltmp2_batch_cell", "ltmp2_batch_set_timing",
                 "ltmp2_batch_get_timing", "ltmp2_real_orbitals",
                 "ltmp2_mlp_forward_noalloc", "ltmp2_get_extrapolation",
                 "ltmp2_direct_hartree", "ltmp2_setup_unrestricted", "ltmp2_setup_kpoints"):
        getattr(lib, name).restype = C.c_int
    lib.ltmp2_supported_grids.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _check(lib, st, ctx=None):
    if st != 0:
        raise LTMP2Error(st, lib.ltmp2_last_error(ctx).decode())


def supported_grids():
    lib = load()
    buf = np.zeros(64, np.int32)
    k = lib.ltmp2_supported_grids(_ptr(buf), 64)
    return [int(x) for x in buf[:k]]


def quadrature(x_min: float, x_max: float, n_tau: int):
    """Host minimax Laplace quadrature (tau, w, delta) from the library."""
    lib = load()
    tau = np.zeros(n_tau)
    w = np.zeros(n_tau)
    d = C.c_double()
    _check(lib, lib.ltmp2_quadrature(x_min, x_max, n_tau, _ptr(tau), _ptr(w), C.byref(d)))
    return tau, w, d.value


def real_orbitals(miller, eps, coeff, n_occ):
    """Host-only: coefficients brought to real form on the grid (complex128 [n_states, n_pw])."""
    lib = load()
    m, e, c = _cell_arrays(miller, eps, coeff)
    out = np.zeros_like(c)
    _check(lib, lib.ltmp2_real_orbitals(m.shape[0], _ptr(m), e.shape[0], _ptr(e), int(n_occ),
                                        _ptr(c), _ptr(out)))
    return out[..., 0] + 1j * out[..., 1]


def _mcheck(lib, st):
    if st != 0:
        raise LTMP2Error(st, lib.ltmp2_mlp_last_error().decode())


def quadrature_table(n_tau, R):
    """Minimax fits (alpha, beta [len(R), n_tau], delta) for ascending R (unit interval)."""
    lib = load()
    R = np.ascontiguousarray(R, np.float64)
    a = np.zeros((len(R), n_tau))
    b = np.zeros((len(R), n_tau))
    d = np.zeros(len(R))
    _mcheck(lib, lib.ltmp2_quadrature_table(n_tau, len(R), _ptr(R), _ptr(a), _ptr(b), _ptr(d)))
    return a, b, d


def mlp_init(seed):
    lib = load()
    p = np.zeros(MLP_NPARAM, np.float32)
    _mcheck(lib, lib.ltmp2_mlp_init(seed, _ptr(p)))
    return p


def mlp_dataset(count, seed, dmin=(0.05, 1.0), ratio=(10.0, 1e4), n_taus=(6, 8, 10, 12)):
    """Seeded training set (X [count, 3], Y [count, 24], M [count, 24], xrange [count, 2])."""
    lib = load()
    X = np.zeros((count, 3), np.float32)
    Y = np.zeros((count, 24), np.float32)
    M = np.zeros((count, 24), np.float32)
    xr = np.zeros((count, 2))
    nt = np.ascontiguousarray(n_taus, np.int32)
    _mcheck(lib, lib.ltmp2_mlp_dataset(count, seed, dmin[0], dmin[1], ratio[0], ratio[1],
                                       _ptr(nt), len(nt), _ptr(X), _ptr(Y), _ptr(M), _ptr(xr)))
    return X, Y, M, xr


def mlp_forward(params, X):
    lib = load()
    X = np.ascontiguousarray(X, np.float32)
    out = np.zeros((X.shape[0], 24), np.float32)
    _mcheck(lib, lib.ltmp2_mlp_forward(_ptr(np.ascontiguousarray(params, np.float32)), _ptr(X),
                                       X.shape[0], _ptr(out), C.c_void_p(_current_stream())))
    return out


MLP_NOALLOC_MAX_ROWS = 16384


def mlp_forward_noalloc(params_dev, X_dev, Y_dev, n=None, stream=None):
    """Network outputs on device tensors (float32: params [5976], X [n, 3], Y [n, 24])
    through the allocation-free entry point; enqueued on the stream, not synchronised."""
    lib = load()
    n = X_dev.shape[0] if n is None else int(n)
    st = _current_stream() if stream is None else stream
    _mcheck(lib, lib.ltmp2_mlp_forward_noalloc(_dptr(params_dev), _dptr(X_dev), n,
                                               _dptr(Y_dev), C.c_void_p(st)))


def mlp_grad(params, X, Y, M):
    lib = load()
    X, Y, M = (np.ascontiguousarray(a, np.float32) for a in (X, Y, M))
    g = np.zeros(MLP_NPARAM, np.float32)
    loss = C.c_float()
    _mcheck(lib, lib.ltmp2_mlp_grad(_ptr(np.ascontiguousarray(params, np.float32)), _ptr(X),
                                    _ptr(Y), _ptr(M), X.shape[0], _ptr(g), C.byref(loss),
                                    C.c_void_p(_current_stream())))
    return g, loss.value


def mlp_train(params, X, Y, M, epochs, batch, lr, seed):
    """Train in place on the GPU; returns the per-epoch loss."""
    lib = load()
    X, Y, M = (np.ascontiguousarray(a, np.float32) for a in (X, Y, M))
    assert params.dtype == np.float32 and params.flags.c_contiguous
    hist = np.zeros(epochs, np.float32)
    _mcheck(lib, lib.ltmp2_mlp_train(_ptr(params), _ptr(X), _ptr(Y), _ptr(M), X.shape[0], epochs,
                                     batch, lr, seed, _ptr(hist), C.c_void_p(_current_stream())))
    return hist


def learned_quadrature(params, x_min, x_max, n_tau, polish_steps=3, cert_tol=1e-6):
    """(tau, w, delta, flags): MLP proposal + Remez polish, certified, else the plain fit."""
    lib = load()
    tau = np.zeros(n_tau)
    w = np.zeros(n_tau)
    d = C.c_double()
    fl = C.c_int()
    _mcheck(lib, lib.ltmp2_learned_quadrature(
        _ptr(np.ascontiguousarray(params, np.float32)), x_min, x_max, n_tau, polish_steps,
        cert_tol, _ptr(tau), _ptr(w), C.byref(d), C.byref(fl), C.c_void_p(_current_stream())))
    return tau, w, d.value, fl.value


def remez_polish(x_min, x_max, tau, w, steps=3, cert_tol=1e-6):
    """Host Remez polish of a proposal: (tau, w, delta, certified)."""
    lib = load()
    tau = np.array(tau, np.float64)
    w = np.array(w, np.float64)
    d = C.c_double()
    ok = C.c_int()
    _mcheck(lib, lib.ltmp2_remez_polish(x_min, x_max, len(tau), steps, cert_tol, _ptr(tau), _ptr(w),
                                        C.byref(d), C.byref(ok)))
    return tau, w, d.value, ok.value


def write_mlp_weights(path, params):
    import struct
    p = np.ascontiguousarray(params, np.float32)
    assert p.size == MLP_NPARAM
    with open(path, "wb") as f:
        f.write(b"LTMP2MLP" + struct.pack("<II", 1, MLP_NPARAM))
        f.write(p.astype("<f4").tobytes())


def read_mlp_weights(path):
    import struct
    raw = open(path, "rb").read()
    if raw[:8] != b"LTMP2MLP":
        raise ValueError("not an LTMP2 MLP weight file")
    ver, cnt = struct.unpack("<II", raw[8:16])
    if ver != 1 or cnt != MLP_NPARAM or len(raw) != 16 + 4 * cnt:
        raise ValueError("unsupported or truncated weight file")
    return np.frombuffer(raw[16:], "<f4").astype(np.float32)


class Context:
    """One prepared cell (ltmp2_setup ... ltmp2_destroy).

    second_spin=(eps_b, coeff_b, n_occ_b) prepares a spin-unrestricted cell
    (ltmp2_setup_unrestricted): eps / coeff / n_occ are then spin channel 1.

    kmesh=n_k prepares the n_k^3 k-point mesh of a cell (ltmp2_setup_kpoints):
    miller and coeff are then lists over the mesh points (per-k Miller
    indices [n_pw_k, 3], complex coefficients [bands, n_pw_k]), eps is
    [n_k^3, bands], n_occ counts bands per k, and energies are per unit cell.
    """

    def __init__(self, L, n_fft, ecut, eaux, miller, eps, coeff, n_occ, n_tau,
                 tau=None, w=None, prec=FP64, workspace_cap=0, stream=None,
                 quad_mode=None, mlp_weights=None, n_extrap=0, extrap_alpha=0.0,
                 second_spin=None, kmesh=None):
        self.lib = load()
        n_pw_k = None
        if kmesh is not None:
            if second_spin is not None:
                raise ValueError("k-point meshes are spin-restricted")
            n_pw_k = np.ascontiguousarray([len(m) for m in miller], np.int32)
            eps = np.asarray(eps, np.float64)
            if eps.ndim != 2 or eps.shape[0] != len(miller) or len(coeff) != len(miller):
                raise ValueError("kmesh: one Miller set, energy row and coefficient block per k")
            nb = eps.shape[1]
            if any(np.asarray(cb).shape[:2] != (nb, len(m)) for cb, m in zip(coeff, miller)):
                raise ValueError("kmesh: coefficients [bands, n_pw_k] per k")
            miller = np.concatenate([np.asarray(m, np.int32) for m in miller])
            coeff = np.concatenate([np.asarray(cb).reshape(-1, *np.asarray(cb).shape[2:])
                                    for cb in coeff])
        miller = np.ascontiguousarray(miller, np.int32)
        eps = np.ascontiguousarray(eps, np.float64)
        coeff = np.asarray(coeff)
        if np.iscomplexobj(coeff):
            coeff = np.stack([coeff.real, coeff.imag], axis=-1)
        coeff = np.ascontiguousarray(coeff, np.float64)
        if quad_mode is None:
            quad_mode = QUAD_GIVEN if tau is not None else (
                QUAD_LEARNED if mlp_weights else QUAD_PLAIN)
        tau_a = None if tau is None else np.ascontiguousarray(tau, np.float64)
        w_a = None if w is None else np.ascontiguousarray(w, np.float64)
        for a in (tau_a, w_a):
            if a is not None and a.shape != (int(n_tau),):
                raise ValueError("tau and w need n_tau entries")
        n_states = eps.shape[-1] if kmesh is not None else eps.shape[0]
        p = Params(float(L), int(n_fft), float(ecut), float(eaux), int(miller.shape[0]),
                   int(n_states), int(n_occ), int(n_tau), int(quad_mode), int(prec),
                   int(workspace_cap), int(n_extrap), float(extrap_alpha))
        if stream is None:
            stream = _current_stream()
        self._ctx = C.c_void_p()
        mw = mlp_weights.encode() if mlp_weights else None
        if kmesh is not None:
            st = self.lib.ltmp2_setup_kpoints(C.byref(p), int(kmesh), _ptr(n_pw_k), _ptr(miller),
                                              _ptr(eps), _ptr(coeff), _ptr(tau_a), _ptr(w_a), mw,
                                              C.c_void_p(stream), C.byref(self._ctx))
        elif second_spin is None:
            st = self.lib.ltmp2_setup(C.byref(p), _ptr(miller), _ptr(eps), _ptr(coeff),
                                      _ptr(tau_a), _ptr(w_a), mw, C.c_void_p(stream),
                                      C.byref(self._ctx))
        else:
            eps_b, coeff_b, n_occ_b = second_spin
            _, eps_b, coeff_b = _cell_arrays(miller, eps_b, coeff_b)
            if eps_b.shape != eps.shape or coeff_b.shape != coeff.shape:
                raise ValueError("both spin channels need the same states and basis")
            st = self.lib.ltmp2_setup_unrestricted(
                C.byref(p), int(n_occ_b), _ptr(miller), _ptr(eps), _ptr(coeff), _ptr(eps_b),
                _ptr(coeff_b), _ptr(tau_a), _ptr(w_a), mw, C.c_void_p(stream),
                C.byref(self._ctx))
        _check(self.lib, st)
        self.info = self.get_info()

    # -- lifetime --
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.ltmp2_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries --
    def get_info(self):
        info = Info()
        _check(self.lib, self.lib.ltmp2_get_info(self._ctx, C.byref(info)), self._ctx)
        return info

    def get_quadrature(self):
        n = self.info.n_tau
        tau = np.zeros(n)
        w = np.zeros(n)
        d = C.c_double()
        _check(self.lib, self.lib.ltmp2_get_quadrature(self._ctx, _ptr(tau), _ptr(w), C.byref(d)),
               self._ctx)
        return tau, w, d.value

    def aux_miller(self):
        out = np.zeros((self.info.n_g, 3), np.int32)
        _check(self.lib, self.lib.ltmp2_aux_miller(self._ctx, _ptr(out)), self._ctx)
        return out

    def set_timing(self, on=True):
        _check(self.lib, self.lib.ltmp2_set_timing(self._ctx, int(on)), self._ctx)

    def get_timing(self):
        """{stage: (ms, launches)} accumulated since set_timing(True)."""
        out = {}
        for k, name in enumerate(STAGES):
            ms = C.c_double()
            n = C.c_long()
            _check(self.lib, self.lib.ltmp2_get_timing(self._ctx, k, C.byref(ms), C.byref(n)),
                   self._ctx)
            out[name] = (ms.value, n.value)
        return out

    # -- the hot path --
    def green(self, itau, row0, nrows, gocc=None, gvir=None):
        """Rows of G_occ / G_vir into torch float64 device tensors [nrows, n_r]."""
        st = self.lib.ltmp2_green(self._ctx, itau, row0, nrows, _dptr(gocc), _dptr(gvir))
        _check(self.lib, st, self._ctx)

    def chi(self, itau, chi_out=None):
        """Unweighted E_d(tau); optional chi(G, G') into a complex128 tensor [n_g, n_g]."""
        e = C.c_double()
        st = self.lib.ltmp2_chi(self._ctx, itau, _dptr(chi_out), C.byref(e))
        _check(self.lib, st, self._ctx)
        return e.value

    def direct_hartree(self, itau):
        """Unweighted E_d(tau) by the Hartree-like route (transformed states)."""
        e = C.c_double()
        st = self.lib.ltmp2_direct_hartree(self._ctx, itau, C.byref(e))
        _check(self.lib, st, self._ctx)
        return e.value

    def exchange(self, itau, g_first=0, g_count=0):
        """Unweighted E_x(tau) over the outer G' range of the half set (0: all)."""
        e = C.c_double()
        st = self.lib.ltmp2_exchange(self._ctx, itau, g_first, g_count, C.byref(e))
        _check(self.lib, st, self._ctx)
        return e.value

    def extrapolation(self, n_extrap):
        """After energy(): (e_aux [n], E_d [n], E_x [n], intercepts (E, E_d, E_x))."""
        ea, ed, ex, ei = (np.zeros(n_extrap), np.zeros(n_extrap), np.zeros(n_extrap),
                          np.zeros(3))
        st = self.lib.ltmp2_get_extrapolation(self._ctx, _ptr(ea), _ptr(ed), _ptr(ex), _ptr(ei))
        _check(self.lib, st, self._ctx)
        return ea, ed, ex, ei

    def energy(self):
        """(E_d, E_x, per_tau [n_tau, 2], quad_err)."""
        ed = C.c_double()
        ex = C.c_double()
        qe = C.c_double()
        pt = np.zeros(2 * self.info.n_tau)
        st = self.lib.ltmp2_energy(self._ctx, C.byref(ed), C.byref(ex), _ptr(pt), C.byref(qe))
        _check(self.lib, st, self._ctx)
        return ed.value, ex.value, pt.reshape(-1, 2), qe.value


def _cell_arrays(miller, eps, coeff):
    miller = np.ascontiguousarray(miller, np.int32)
    eps = np.ascontiguousarray(eps, np.float64)
    coeff = np.asarray(coeff)
    if np.iscomplexobj(coeff):
        coeff = np.stack([coeff.real, coeff.imag], axis=-1)
    return miller, eps, np.ascontiguousarray(coeff, np.float64)


class Batch:
    """Many independent cells evaluated together (ltmp2_batch_* calls).

    cells: sequence of dicts with keys L, n_fft, ecut, eaux, miller, eps,
    coeff, n_occ, n_tau and optionally tau, w (a given quadrature).
    """

    def __init__(self, cells, prec=FP64, mlp_weights=None, stream=None):
        self.lib = load()
        n = len(cells)
        params = (Params * n)()
        keep = []
        ptrs = {k: (C.c_void_p * n)() for k in ("m", "e", "c", "t", "w")}
        any_given = False
        for k, cell in enumerate(cells):
            m, e, c = _cell_arrays(cell["miller"], cell["eps"], cell["coeff"])
            t = cell.get("tau")
            w = cell.get("w")
            t = None if t is None else np.ascontiguousarray(t, np.float64)
            w = None if w is None else np.ascontiguousarray(w, np.float64)
            any_given |= t is not None
            mode = QUAD_GIVEN if t is not None else (QUAD_LEARNED if mlp_weights else QUAD_PLAIN)
            params[k] = Params(float(cell["L"]), int(cell["n_fft"]), float(cell["ecut"]),
                               float(cell["eaux"]), int(m.shape[0]), int(e.shape[0]),
                               int(cell["n_occ"]), int(cell["n_tau"]), mode, int(prec), 0)
            keep += [m, e, c, t, w]
            for key, a in zip("mectw", (m, e, c, t, w)):
                ptrs[key][k] = None if a is None else a.ctypes.data
        if stream is None:
            stream = _current_stream()
        self._b = C.c_void_p()
        st = self.lib.ltmp2_batch_create(
            n, C.cast(params, C.c_void_p), C.cast(ptrs["m"], C.c_void_p),
            C.cast(ptrs["e"], C.c_void_p), C.cast(ptrs["c"], C.c_void_p),
            C.cast(ptrs["t"], C.c_void_p) if any_given else None,
            C.cast(ptrs["w"], C.c_void_p) if any_given else None,
            mlp_weights.encode() if mlp_weights else None, C.c_void_p(stream), C.byref(self._b))
        del keep
        self._bcheck(st, None)
        self.n_cells = n

    def _bcheck(self, st, b):
        if st != 0:
            raise LTMP2Error(st, self.lib.ltmp2_batch_last_error(b).decode())

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            self.lib.ltmp2_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def energy(self):
        """(E_d [n_cells], E_x [n_cells])."""
        ed = np.zeros(self.n_cells)
        ex = np.zeros(self.n_cells)
        self._bcheck(self.lib.ltmp2_batch_energy(self._b, _ptr(ed), _ptr(ex)), self._b)
        return ed, ex

    def stats(self):
        s = BatchStats()
        self._bcheck(self.lib.ltmp2_batch_info(self._b, C.byref(s)), self._b)
        return s

    def group(self, g):
        """dict of grid size, cells, rounds, slab_tile, wg_per_cu, tuned_ms of group g."""
        v = [C.c_int() for _ in range(5)]
        ms = C.c_double()
        self._bcheck(self.lib.ltmp2_batch_group(self._b, int(g), *[C.byref(x) for x in v],
                                                C.byref(ms)), self._b)
        return dict(zip(("n_fft", "n_cells", "rounds", "slab_tile", "wg_per_cu"),
                        (x.value for x in v)), tuned_ms=ms.value)

    def set_timing(self, on=True):
        self._bcheck(self.lib.ltmp2_batch_set_timing(self._b, int(on)), self._b)

    def get_timing(self):
        """{stage: (ms, launches)} accumulated since set_timing(True)."""
        out = {}
        for k, name in enumerate(STAGES):
            ms = C.c_double()
            n = C.c_long()
            self._bcheck(self.lib.ltmp2_batch_get_timing(self._b, k, C.byref(ms), C.byref(n)),
                         self._b)
            out[name] = (ms.value, n.value)
        return out

    def cell_info(self, k):
        info = Info()
        self._bcheck(self.lib.ltmp2_batch_cell(self._b, int(k), C.byref(info)), self._b)
        return info


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device output must be a contiguous GPU tensor")
    return C.c_void_p(t.data_ptr())


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return 0
