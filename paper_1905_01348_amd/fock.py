"""ctypes binding of libfock's C ABI (include/fock.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch tensors supply device memory and streams.  If libfock.so has
not been built the binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfock.so")

# ---- enums (mirror include/fock.h) -----------------------------------------
FX_OK = 0
FX_ERR_INVALID = -1
FX_ERR_UNSUPPORTED = -2
FX_ERR_OOM = -3
FX_ERR_NOT_POSDEF = -4
FX_ERR_DEVICE = -5
FX_ERR_BUSY = -6
FX_ERR_CANCELLED = -7
STATUS_NAMES = {0: "FX_OK", -1: "FX_ERR_INVALID", -2: "FX_ERR_UNSUPPORTED", -3: "FX_ERR_OOM",
                -4: "FX_ERR_NOT_POSDEF", -5: "FX_ERR_DEVICE", -6: "FX_ERR_BUSY", -7: "FX_ERR_CANCELLED"}

FX_C128, FX_C64 = 0, 1
FX_COULOMB, FX_HSE = 0, 1
PREC = {
    "fp64": 0, "fp32": 1, "fp32acc64": 2,
    "ace_fp64": 3, "ace_fp32r": 4, "ace_bf16r": 5, "ace_fp32": 6, "ace_bf16": 7, "ace_fp16r": 8, "ace_fp16": 9,
}
KIND = {"coulomb": FX_COULOMB, "hse": FX_HSE}
KERNEL_IDS = {"vx_plane_fwd": 0, "vx_pencil_z": 1, "vx_plane_inv": 2, "convert": 3, "gemm_cn": 4, "gemm_nn": 5,
              "reduce": 6, "split": 7, "linalg": 8}


class FxCell(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("len", C.c_double * 3)]


class FxKernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("omega", C.c_double), ("scale", C.c_double)]


class FxServeCfg(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("n_streams", C.c_int32), ("max_batch_pairs", C.c_int32),
                ("hbm_budget_bytes", C.c_size_t), ("autotune", C.c_int32), ("autotune_targets", C.c_int32),
                ("vx_work_mb", C.c_int32), ("max_queue", C.c_int32)]


class FxRequest(C.Structure):
    _fields_ = [("traj", C.c_int32), ("op", C.c_int32), ("first", C.c_int32), ("count", C.c_int32),
                ("t_arrival_s", C.c_double), ("out", C.c_void_p), ("ld_out", C.c_int64)]


class FxServeReport(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
                ("req_per_s", C.c_double), ("pairs_per_s", C.c_double), ("busy_frac", C.c_double),
                ("wall_s", C.c_double), ("n_done", C.c_int64), ("n_rejected", C.c_int64),
                ("n_batches", C.c_int64), ("hbm_peak_bytes", C.c_size_t), ("n_cancelled", C.c_int64)]


class FxVxConfig(C.Structure):
    _fields_ = [("kernels", C.c_int32), ("work_mb", C.c_int32), ("a_prefetch", C.c_int32),
                ("b_variant", C.c_int32), ("c_variant", C.c_int32), ("a_variant", C.c_int32), ("nt_hint", C.c_int32),
                ("b_xtile", C.c_int32), ("b_threads", C.c_int32),
                ("radix", (C.c_int32 * 4) * 3), ("c_split", C.c_int32)]


def config_to_dict(c):
    return {"kernels": c.kernels, "work_mb": c.work_mb, "a_prefetch": c.a_prefetch, "b_variant": c.b_variant,
            "c_variant": c.c_variant, "a_variant": c.a_variant, "nt_hint": c.nt_hint, "b_xtile": c.b_xtile,
            "b_threads": c.b_threads, "radix": [list(row) for row in c.radix], "c_split": c.c_split}


def config_from_dict(d):
    c = FxVxConfig()
    c.a_prefetch = -1
    c.nt_hint = -1
    for k in ("kernels", "work_mb", "a_prefetch", "b_variant", "c_variant", "a_variant", "nt_hint", "b_xtile",
              "b_threads", "c_split"):
        if k in d:
            setattr(c, k, int(d[k]))
    for a, row in enumerate(d.get("radix", [])):
        for i, r in enumerate(list(row) + [0] * (4 - len(row))):
            c.radix[a][i] = int(r)
    return c


# exported names and their signatures
_SIGS = {
    "fx_init": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]),
    "fx_finalize": (C.c_int, [C.c_void_p]),
    "fx_last_error": (C.c_char_p, []),
    "fx_version": (C.c_char_p, []),
    "fx_memory": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "fx_apply_vx": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.POINTER(FxKernel),
                              C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_int64,
                              C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "fx_apply_vx_noalloc": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.POINTER(FxKernel),
                                      C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32, C.c_int64,
                                      C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "fx_build_ace": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.POINTER(FxKernel),
                               C.c_void_p, C.c_int32, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_void_p,
                               C.POINTER(C.c_void_p), C.c_void_p]),
    "fx_apply_ace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64,
                               C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "fx_ace_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fx_ace_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "fx_ace_free": (C.c_int, [C.c_void_p]),
    "fx_serve_create": (C.c_int, [C.c_void_p, C.POINTER(FxServeCfg), C.POINTER(C.c_void_p)]),
    "fx_serve_register": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(FxCell), C.POINTER(FxKernel),
                                    C.c_void_p, C.c_int32, C.c_int64, C.c_int, C.c_int, C.c_int]),
    "fx_serve": (C.c_int, [C.c_void_p, C.POINTER(FxRequest), C.c_int32, C.POINTER(C.c_int),
                           C.POINTER(C.c_double), C.POINTER(FxServeReport)]),
    "fx_serve_destroy": (C.c_int, [C.c_void_p]),
    "fx_serve_cancel": (C.c_int, [C.c_void_p, C.c_int32]),
    "fx_vx_load_configs": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int32)]),
    "fx_vx_save_configs": (C.c_int, [C.c_void_p, C.c_char_p]),
    "fx_graph_cache": (C.c_int, [C.c_void_p, C.c_int32]),
    "fx_graph_cache_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32)]),
    "fx_prof_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "fx_prof_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
    "fx_debug_host_pair": (C.c_int, [C.POINTER(FxCell), C.POINTER(FxKernel), C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "fx_debug_host_pair_plan": (C.c_int, [C.POINTER(FxCell), C.POINTER(FxKernel), C.c_int, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p]),
    "fx_debug_axis_plans": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_int32)]),
    "fx_debug_fail_alloc": (C.c_int, [C.c_int64]),
    "fx_debug_stream": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_double)]),
    "fx_apply_kinetic": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.c_void_p, C.c_int32, C.c_int64, C.c_void_p,
                                   C.c_int64, C.c_int, C.c_int, C.c_void_p]),
    "fx_pt_residual": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.POINTER(FxKernel), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int32, C.c_int64, C.c_int, C.c_double, C.c_int, C.c_int32, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p]),
    "fx_orthonormalize": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int, C.c_void_p]),
    "fx_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int, C.c_void_p,
                             C.c_void_p, C.c_void_p]),
    "fx_vx_autotune": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.POINTER(FxKernel), C.c_int32, C.c_int32, C.c_int32,
                                 C.c_int, C.c_void_p, C.POINTER(FxVxConfig), C.POINTER(C.c_double)]),
    "fx_vx_set_config": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.c_int, C.c_int32, C.POINTER(FxVxConfig)]),
    "fx_vx_get_config": (C.c_int, [C.c_void_p, C.POINTER(FxCell), C.c_int, C.c_int32, C.POINTER(FxVxConfig),
                                   C.POINTER(C.c_int32)]),
}

_lib = None


def load():
    """Load libfock.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfock.so not built ({LIB_PATH}); run python -m paper_1905_01348_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FockError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status):
    if status != FX_OK:
        raise FockError(status, load().fx_last_error().decode(errors="replace"))


def make_cell(n, L):
    n3 = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n, n, n)))
    l3 = tuple(float(v) for v in (L if hasattr(L, "__len__") else (L, L, L)))
    c = FxCell()
    c.n[:] = n3
    c.len[:] = l3
    return c


def make_kernel(kind="hse", omega=0.106, scale=1.0):
    k = FxKernel()
    k.kind = KIND[kind] if isinstance(kind, str) else int(kind)
    k.omega = float(omega)
    k.scale = float(scale)
    return k


def _dtype_code(t):
    import torch

    if t.dtype == torch.complex128:
        return FX_C128
    if t.dtype == torch.complex64:
        return FX_C64
    raise TypeError(f"orbitals must be complex64 or complex128, got {t.dtype}")


def _cols(t, nr):
    """(pointer, ncols, ld) of a device tensor holding columns of nr points."""
    if not t.is_cuda:
        raise TypeError("device (cuda/hip) tensor expected")
    if t.dim() == 1:
        if t.numel() != nr:
            raise ValueError("1-D tensor must hold one orbital")
        return t.data_ptr(), 1, nr
    if t.stride(-1) != 1:
        raise ValueError("innermost dimension must be contiguous")
    flat_inner = 1
    for s in t.shape[1:]:
        flat_inner *= s
    if flat_inner != nr:
        raise ValueError(f"each column must hold N_r = {nr} points, got {flat_inner}")
    # every dim but the first must be contiguous within a column
    expect = 1
    for d in range(t.dim() - 1, 0, -1):
        if t.stride(d) != expect and t.shape[d] != 1:
            raise ValueError("columns must be contiguous")
        expect *= t.shape[d]
    return t.data_ptr(), t.shape[0], t.stride(0)


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """One libfock context on one device (owns tables, workspaces, budget)."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        lib = load()
        h = C.c_void_p()
        _check(lib.fx_init(int(device), int(hbm_budget_bytes), C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            _check(load().fx_finalize(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def memory(self):
        a, b = C.c_size_t(), C.c_size_t()
        _check(load().fx_memory(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- per-kernel timing (include/fock_prof.h) --------------------------------
    def prof_enable(self, on=True):
        _check(load().fx_prof_enable(self.h, 1 if on else 0))

    def prof_read(self, kid):
        """(launches, total_ms, algorithmic work: bytes or executed flops) of one kernel id."""
        n, ms, wk = C.c_int64(), C.c_double(), C.c_double()
        _check(load().fx_prof_read(self.h, int(kid), C.byref(n), C.byref(ms), C.byref(wk)))
        return n.value, ms.value, wk.value

    # -- V_X ------------------------------------------------------------------
    def apply_vx(self, psi, phi=None, *, n, L, kernel="hse", omega=0.106, scale=1.0, prec="fp32acc64",
                 out=None, out_dtype=None, stream=None, energy=False):
        """out = V_X[psi] phi; returns out (and E_X as a 0-d float64 tensor if energy)."""
        import torch

        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        kern = make_kernel(kernel, omega, scale)
        if phi is None:
            phi = psi
        pp, npsi, ldp = _cols(psi, nr)
        fp, nphi, ldf = _cols(phi, nr)
        if out is None:
            od = out_dtype or (torch.complex128 if prec in ("fp64", "fp32acc64") else torch.complex64)
            out = torch.empty((nphi,) + tuple(phi.shape[1:]), dtype=od, device=phi.device)
        op, nout, ldo = _cols(out, nr)
        if nout != nphi:
            raise ValueError("out must have as many columns as phi")
        if psi.dtype != phi.dtype:
            raise TypeError("psi and phi must have the same dtype")
        ex = torch.zeros((), dtype=torch.float64, device=psi.device) if energy else None
        _check(load().fx_apply_vx(self.h, C.byref(cell), C.byref(kern), pp, npsi, ldp, fp, nphi, ldf, op, ldo,
                                  _dtype_code(psi), _dtype_code(out), PREC[prec], _stream_ptr(stream),
                                  C.c_void_p(ex.data_ptr()) if ex is not None else None))
        return (out, ex) if energy else out

    def apply_vx_noalloc(self, psi, phi=None, *, out, n, L, kernel="hse", omega=0.106, scale=1.0,
                         prec="fp32acc64", stream=None, energy_out=None):
        """out = V_X[psi] phi through fx_apply_vx_noalloc (no device allocation in the library;
        out and the optional float64 device scalar energy_out are the caller's).  Returns out."""
        import torch

        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        kern = make_kernel(kernel, omega, scale)
        if phi is None:
            phi = psi
        pp, npsi, ldp = _cols(psi, nr)
        fp, nphi, ldf = _cols(phi, nr)
        op, nout, ldo = _cols(out, nr)
        if nout != nphi:
            raise ValueError("out must have as many columns as phi")
        if psi.dtype != phi.dtype:
            raise TypeError("psi and phi must have the same dtype")
        ep = None
        if energy_out is not None:
            if energy_out.dtype != torch.float64 or energy_out.numel() != 1 or not energy_out.is_cuda:
                raise ValueError("energy_out must be a one-element float64 device tensor")
            ep = C.c_void_p(energy_out.data_ptr())
        _check(load().fx_apply_vx_noalloc(self.h, C.byref(cell), C.byref(kern), pp, npsi, ldp, fp, nphi, ldf, op,
                                          ldo, _dtype_code(psi), _dtype_code(out), PREC[prec], _stream_ptr(stream),
                                          ep))
        return out

    def debug_stream(self, buf, mode, *, iters=5, stream=None):
        """GB/s of a read (mode 0), write (1) or in-place (2) stream over the device tensor buf."""
        out = C.c_double()
        _check(load().fx_debug_stream(self.h, int(mode), C.c_void_p(buf.data_ptr()),
                                      buf.numel() * buf.element_size(), int(iters), _stream_ptr(stream),
                                      C.byref(out)))
        return out.value

    # -- end-of-step operations ----------------------------------------------------
    def apply_kinetic(self, phi, *, n, L, out=None, out_dtype=None, stream=None):
        """out = -(1/2) Laplacian phi on the periodic grid (|G|^2/2 on each planewave), FP64."""
        import torch

        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        fp, nphi, ldf = _cols(phi, nr)
        if out is None:
            out = torch.empty((nphi,) + tuple(phi.shape[1:]), dtype=out_dtype or phi.dtype, device=phi.device)
        op, nout, ldo = _cols(out, nr)
        if nout != nphi:
            raise ValueError("out must have as many columns as phi")
        _check(load().fx_apply_kinetic(self.h, C.byref(cell), fp, nphi, ldf, op, ldo, _dtype_code(phi),
                                       _dtype_code(out), _stream_ptr(stream)))
        return out

    def pt_residual(self, psi, psi_half, *, n, L, hpsi=None, dt, kernel="hse", omega=0.106, scale=1.0,
                    vx_prec="fp32acc64", kinetic=False, out=None, s_out=None, stream=None):
        """R = Psi + (i dt/2)(H Psi - Psi S) - Psi_half with S = Psi^H H Psi; H = V_X if hpsi is None,
        plus -(1/2) Laplacian if kinetic."""
        import torch

        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        kern = make_kernel(kernel, omega, scale)
        pp, npsi, ldp = _cols(psi, nr)
        fp, nf, ldf = _cols(psi_half, nr)
        if nf != npsi or ldf != ldp or psi_half.dtype != psi.dtype:
            raise ValueError("psi_half must have psi's shape, stride and dtype")
        hp = None
        if hpsi is not None:
            hp, nh, ldh = _cols(hpsi, nr)
            if nh != npsi or ldh != ldp or hpsi.dtype != psi.dtype:
                raise ValueError("hpsi must have psi's shape, stride and dtype")
        if out is None:
            out = torch.empty_like(psi)
        op, no, ldo = _cols(out, nr)
        if no != npsi or out.dtype != psi.dtype:
            raise ValueError("out must have psi's column count and dtype")
        sp = None
        if s_out is not None:
            if s_out.dtype != torch.complex128 or s_out.numel() != npsi * npsi or not s_out.is_contiguous():
                raise ValueError("s_out must be a contiguous complex128 tensor of n x n")
            sp = C.c_void_p(s_out.data_ptr())
        _check(load().fx_pt_residual(self.h, C.byref(cell), C.byref(kern), pp, hp, fp, npsi, ldp, _dtype_code(psi),
                                     float(dt), PREC[vx_prec], 1 if kinetic else 0, op, ldo, sp,
                                     _stream_ptr(stream)))
        return out

    def orthonormalize(self, psi, *, stream=None):
        """Cholesky-QR re-orthonormalisation of the columns of psi, in place; returns psi."""
        nr = int(psi[0].numel())
        pp, npsi, ldp = _cols(psi, nr)
        _check(load().fx_orthonormalize(self.h, pp, npsi, ldp, nr, _dtype_code(psi), _stream_ptr(stream)))
        return psi

    def density(self, psi, *, occ=None, out=None, stream=None):
        """rho(r) = sum_i f_i |psi_i(r)|^2 in FP64 (shape of one orbital)."""
        import torch

        nr = int(psi[0].numel())
        pp, npsi, ldp = _cols(psi, nr)
        if out is None:
            out = torch.empty(tuple(psi.shape[1:]), dtype=torch.float64, device=psi.device)
        if out.dtype != torch.float64 or out.numel() != nr or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of N_r elements")
        oc = None
        if occ is not None:
            if occ.dtype != torch.float64 or occ.numel() != npsi or not occ.is_contiguous():
                raise ValueError("occ must be a contiguous float64 tensor of n elements")
            oc = C.c_void_p(occ.data_ptr())
        _check(load().fx_density(self.h, pp, npsi, ldp, nr, _dtype_code(psi), oc, C.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream)))
        return out

    # -- launch configuration of the V_X path ------------------------------------
    def vx_autotune(self, *, n, L, n_psi, n_phi, phi_is_psi=False, prec="fp32acc64", kernel="hse", omega=0.106,
                    scale=1.0, stream=None):
        """Tune and store the V_X launch configuration of this shape; returns (config dict, ms per 1000 pairs)."""
        cell = make_cell(n, L)
        kern = make_kernel(kernel, omega, scale)
        cfg = FxVxConfig()
        ms = C.c_double()
        _check(load().fx_vx_autotune(self.h, C.byref(cell), C.byref(kern), int(n_psi), int(n_phi),
                                     1 if phi_is_psi else 0, PREC[prec], _stream_ptr(stream), C.byref(cfg),
                                     C.byref(ms)))
        return config_to_dict(cfg), ms.value

    def set_vx_config(self, cfg, *, n, L=1.0, prec="fp32acc64", phi_is_psi=False):
        """Store a configuration (dict, fields of fx_vx_config) for (grid, prec, form); None clears it."""
        cell = make_cell(n, L)
        c = config_from_dict(cfg) if cfg is not None else None
        _check(load().fx_vx_set_config(self.h, C.byref(cell), PREC[prec], 1 if phi_is_psi else 0,
                                       C.byref(c) if c is not None else None))

    def get_vx_config(self, *, n, L=1.0, prec="fp32acc64", phi_is_psi=False):
        """(config dict, is_set) stored for (grid, prec, form)."""
        cell = make_cell(n, L)
        c = FxVxConfig()
        is_set = C.c_int32()
        _check(load().fx_vx_get_config(self.h, C.byref(cell), PREC[prec], 1 if phi_is_psi else 0, C.byref(c),
                                       C.byref(is_set)))
        return config_to_dict(c), bool(is_set.value)

    def load_configs(self, path):
        """Load the launch configurations of this kind of device from a file; returns how many."""
        n = C.c_int32()
        _check(load().fx_vx_load_configs(self.h, os.fsencode(path), C.byref(n)))
        return n.value

    def save_configs(self, path):
        """Save the context's launch configurations to a file (other devices' lines are kept)."""
        _check(load().fx_vx_save_configs(self.h, os.fsencode(path)))

    # -- replay cache ------------------------------------------------------------
    def graph_cache(self, max_entries):
        """Replay cache of apply_vx / Ace.apply calls (0 turns it off)."""
        _check(load().fx_graph_cache(self.h, int(max_entries)))

    def graph_cache_stats(self):
        """(hits, misses, entries) of the replay cache."""
        h, m, e = C.c_int64(), C.c_int64(), C.c_int32()
        _check(load().fx_graph_cache_stats(self.h, C.byref(h), C.byref(m), C.byref(e)))
        return h.value, m.value, e.value

    # -- ACE ------------------------------------------------------------------
    def build_ace(self, psi, *, n, L, kernel="hse", omega=0.106, scale=1.0, vx_prec="fp64",
                  ace_prec="ace_fp64", stream=None):
        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        kern = make_kernel(kernel, omega, scale)
        import torch

        pp, npsi, ldp = _cols(psi, nr)
        h = C.c_void_p()
        ex = torch.zeros((), dtype=torch.float64, device=psi.device)
        _check(load().fx_build_ace(self.h, C.byref(cell), C.byref(kern), pp, npsi, ldp, _dtype_code(psi),
                                   PREC[vx_prec], PREC[ace_prec], _stream_ptr(stream), C.byref(h),
                                   C.c_void_p(ex.data_ptr())))
        # the build has already waited on its stream (Cholesky status); E_X is on the device
        return Ace(self, h, nr, npsi, tuple(psi.shape[1:]), float(ex.item()), psi.device)


class Ace:
    """Handle of ACE factors built by Context.build_ace."""

    def __init__(self, ctx, h, nr, n, grid_shape, ex, device):
        self.ctx, self.h, self.nr, self.n, self.grid_shape, self.ex, self.device = ctx, h, nr, n, grid_shape, ex, device

    def apply(self, phi, *, prec="ace_fp64", out=None, out_dtype=None, stream=None):
        import torch

        fp, nphi, ldf = _cols(phi, self.nr)
        if out is None:
            out = torch.empty((nphi,) + tuple(phi.shape[1:]), dtype=out_dtype or phi.dtype, device=phi.device)
        op, nout, ldo = _cols(out, self.nr)
        if nout != nphi:
            raise ValueError("out must have as many columns as phi")
        _check(load().fx_apply_ace(self.ctx.h, self.h, fp, nphi, ldf, op, ldo, _dtype_code(phi), _dtype_code(out),
                                   PREC[prec], _stream_ptr(stream)))
        return out

    def export(self):
        import torch

        xi = torch.empty((self.n, self.nr), dtype=torch.complex128, device=self.device)
        L = torch.empty((self.n, self.n), dtype=torch.complex128, device=self.device)
        M = torch.empty((self.n, self.n), dtype=torch.complex128, device=self.device)
        _check(load().fx_ace_export(self.h, xi.data_ptr(), L.data_ptr(), M.data_ptr()))
        # L and M are column-major N x N: the torch view (col, row) -> transpose
        return xi, L.T.contiguous(), M.T.contiguous()

    def free(self):
        if self.h:
            _check(load().fx_ace_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching server over resident trajectories (fx_serve_*)."""

    def __init__(self, ctx, max_slots=8, n_streams=4, max_batch_pairs=1 << 16, hbm_budget_bytes=0, autotune=False,
                 autotune_targets=8, vx_work_mb=0, max_queue=0):
        cfg = FxServeCfg()
        cfg.max_slots, cfg.n_streams, cfg.max_batch_pairs = int(max_slots), int(n_streams), int(max_batch_pairs)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.autotune, cfg.autotune_targets = (1 if autotune else 0), int(autotune_targets)
        cfg.vx_work_mb = int(vx_work_mb)
        cfg.max_queue = int(max_queue)
        h = C.c_void_p()
        _check(load().fx_serve_create(ctx.h, C.byref(cfg), C.byref(h)))
        self.ctx, self.h = ctx, h
        self.trajs = {}

    def register(self, traj, psi, *, n, L, kernel="hse", omega=0.106, scale=1.0, vx_prec="fp32acc64",
                 ace_prec="ace_fp32r"):
        cell = make_cell(n, L)
        nr = cell.n[0] * cell.n[1] * cell.n[2]
        kern = make_kernel(kernel, omega, scale)
        pp, npsi, ldp = _cols(psi, nr)
        _check(load().fx_serve_register(self.h, int(traj), C.byref(cell), C.byref(kern), pp, npsi, ldp,
                                        _dtype_code(psi), PREC[vx_prec], PREC[ace_prec]))
        self.trajs[traj] = (nr, npsi, psi.dtype)

    def serve(self, requests):
        """requests: list of dicts(traj, op, first, count, t, out).  Returns (status, latency_ms, report dict)."""
        n = len(requests)
        arr = (FxRequest * max(n, 1))()
        for i, r in enumerate(requests):
            o = r["out"]
            if o is None:
                op_, ld = None, 0
            elif r["traj"] in self.trajs:
                nr_t, _, dt_t = self.trajs[r["traj"]]
                op_, ncol, ld = _cols(o, nr_t)
                # the library writes `count` columns of the trajectory's dtype at ld
                if o.dtype != dt_t:
                    raise ValueError(f"request {i}: out must have the trajectory's dtype {dt_t}")
                if ncol < int(r["count"]):
                    raise ValueError(f"request {i}: out holds {ncol} columns, the request writes {r['count']}")
            else:  # unknown trajectory: the library reports it per request
                op_, ld = o.data_ptr(), o.stride(0)
            arr[i].traj, arr[i].op, arr[i].first, arr[i].count = r["traj"], r["op"], r["first"], r["count"]
            arr[i].t_arrival_s = float(r["t"])
            arr[i].out = op_
            arr[i].ld_out = ld
        st = (C.c_int * max(n, 1))()
        lat = (C.c_double * max(n, 1))()
        rep = FxServeReport()
        _check(load().fx_serve(self.h, arr, n, st, lat, C.byref(rep)))
        report = {f: getattr(rep, f) for f, _ in FxServeReport._fields_}
        return [st[i] for i in range(n)], [lat[i] for i in range(n)], report

    def cancel(self, index):
        """Cancel request `index` of the running (or next) serve call; thread-safe."""
        _check(load().fx_serve_cancel(self.h, int(index)))

    def close(self):
        if self.h:
            _check(load().fx_serve_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_host_pair(psi_j, phi_k, *, n, L, kernel="hse", omega=0.106, scale=1.0, prec=0, radix=None):
    """Run the library's pass code on the host for one pair (prec 0: FP64, 1: FP32), optionally
    with a radix schedule per axis (3 rows, stages in order, [] or zeros for the default)."""
    import numpy as np

    cell = make_cell(n, L)
    kern = make_kernel(kernel, omega, scale)
    a = np.ascontiguousarray(psi_j, dtype=np.complex128)
    b = np.ascontiguousarray(phi_k, dtype=np.complex128)
    v = np.empty_like(a)
    if radix is None:
        _check(load().fx_debug_host_pair(C.byref(cell), C.byref(kern), int(prec), a.ctypes.data, b.ctypes.data,
                                         v.ctypes.data))
    else:
        r = np.zeros((3, 4), dtype=np.int32)
        for ax, row in enumerate(radix):
            r[ax, :len(row)] = row
        _check(load().fx_debug_host_pair_plan(C.byref(cell), C.byref(kern), int(prec), r.ctypes.data, a.ctypes.data,
                                              b.ctypes.data, v.ctypes.data))
    return v


def debug_fail_alloc(k):
    """Make the k-th device allocation of the library from now fail once with FX_ERR_OOM (0 cancels)."""
    _check(load().fx_debug_fail_alloc(int(k)))


def debug_axis_plans(n, max_plans=6):
    """The radix schedules the autotuner considers for edge n (default first), as lists."""
    import numpy as np

    out = np.zeros((max_plans, 4), dtype=np.int32)
    cnt = C.c_int32()
    _check(load().fx_debug_axis_plans(int(n), int(max_plans), out.ctypes.data, C.byref(cnt)))
    return [[int(r) for r in row if r] for row in out[:cnt.value]]
