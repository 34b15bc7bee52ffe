"""Thin ctypes binding of libvp (C ABI in include/vp.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Functions keep the C names; arrays are torch CUDA float64 tensors whose shapes
and placement are checked here before any kernel is launched.  If the library
is missing the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libvp.so")

VP_OK, VP_NOT_CONVERGED, VP_LINESEARCH_FAIL, VP_KRYLOV_MAXIT = 0, 1, 2, 3
VP_EINVAL, VP_EHIP, VP_ENOMEM, VP_ESTATE, VP_ENONFINITE, VP_EBREAKDOWN = -1, -2, -3, -4, -5, -6
VP_SVN, VP_STDN = 0, 1
VP_PREC_FP64, VP_PREC_FP32, VP_PREC_FP32_BF16COARSE, VP_PREC_BF16, VP_PREC_FP16_BF16COARSE, VP_PREC_FP16 = \
    0, 1, 2, 3, 4, 5
VP_PREC_FP16_FP32COARSE = 6
VP_KRYLOV_FGMRES, VP_KRYLOV_FCG = 0, 1
VP_LS_ENERGY, VP_LS_RESIDUAL = 0, 1
VP_AMG_SA, VP_AMG_RS = 0, 1
VP_AMG_VAR_NO_TAIL, VP_AMG_VAR_NO_PAIRS, VP_AMG_VAR_NO_TAIL_LDS, VP_AMG_VAR_NO_P16 = 1, 2, 4, 8
VPNET_START_LEARNED, VPNET_START_PREVIOUS, VPNET_START_ZERO = 1, 2, 4
VPNET_MAX_POOL = 8
VPNET_POOLED_SCALE = 0.3
START = {"learned": VPNET_START_LEARNED, "previous": VPNET_START_PREVIOUS, "zero": VPNET_START_ZERO}

EXPORTED = ["vp_create", "vp_destroy", "vp_last_error", "vp_set_state", "vp_residual",
            "vp_newton_assemble", "vp_operator_apply", "vp_operator_export", "vp_amg_setup",
            "vp_amg_apply", "vp_amg_info", "vp_amg_export", "vp_amg_rs_info", "vp_amg_rs_export",
            "vp_krylov_solve", "vp_krylov_solve_noalloc", "vp_pi_update", "vp_pi_init",
            "vp_newton_step", "vp_newton_solve", "vp_default_opts", "vp_advect", "vp_profile",
            "vp_profile_read"]
EXPORTED_NET = ["vpnet_create", "vpnet_destroy", "vpnet_last_error", "vpnet_param_count",
                "vpnet_set_params", "vpnet_get_params", "vpnet_get_grads", "vpnet_forward",
                "vpnet_backward", "vpnet_adam", "vpnet_train_step", "vpnet_features",
                "vpnet_targets", "vpnet_guess", "vpnet_infer", "vpnet_inspect", "vpnet_gemm"]
VP_KID = dict(apply_fine=0, cheb_step0=1, sten_resid0=2, residual=3, assemble=4, vcycle=5, cheb_pair0=6,
              cheb_walk4=7)


class vp_problem_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("rho_ice", C.c_double), ("rho_air", C.c_double), ("rho_ocean", C.c_double),
                ("C_air", C.c_double), ("C_ocean", C.c_double), ("P_star", C.c_double),
                ("C_strength", C.c_double), ("e_ratio", C.c_double), ("f_coriolis", C.c_double),
                ("dt", C.c_double), ("delta_min", C.c_double), ("order", C.c_int32)]


class vp_amg_opts(C.Structure):
    _fields_ = [("cheb_degree", C.c_int), ("max_coarse", C.c_int), ("precision", C.c_int),
                ("cheb_ratio", C.c_double), ("omega_scale", C.c_double), ("kind", C.c_int), ("sweeps", C.c_int),
                ("strong_threshold", C.c_double), ("max_row_sum", C.c_double), ("variant", C.c_int),
                ("walk4_rows", C.c_int)]


class vp_krylov_opts(C.Structure):
    _fields_ = [("method", C.c_int), ("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double)]


class vp_krylov_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_resid", C.c_double)]


class vp_newton_opts(C.Structure):
    _fields_ = [("variant", C.c_int), ("tol", C.c_double), ("eta_max", C.c_double),
                ("max_backtracks", C.c_int), ("ls_mode", C.c_int)]


class vp_newton_info(C.Structure):
    _fields_ = [("rnorm", C.c_double), ("rnorm0", C.c_double), ("rnorm_new", C.c_double),
                ("energy", C.c_double), ("energy_new", C.c_double), ("alpha", C.c_double),
                ("eta", C.c_double), ("backtracks", C.c_int), ("krylov_iters", C.c_int)]


class vp_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("krylov_iters", C.c_int), ("rnorm0", C.c_double),
                ("rel_resid", C.c_double)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libvp.so not built at {_LIB_PATH}; run __graft_entry__.build()")
    lib = C.CDLL(_LIB_PATH)
    P, D, I = C.c_void_p, C.c_double, C.c_int
    sig = {
        "vp_create": (I, [C.POINTER(vp_problem_desc), P, C.POINTER(P)]),
        "vp_destroy": (None, [P]),
        "vp_last_error": (C.c_char_p, [P]),
        "vp_set_state": (I, [P, P, P, P, P, P]),
        "vp_residual": (I, [P, P, P, C.POINTER(D), C.POINTER(D)]),
        "vp_newton_assemble": (I, [P, P, P, I]),
        "vp_operator_apply": (I, [P, P, P]),
        "vp_operator_export": (I, [P, P]),
        "vp_amg_setup": (I, [P, C.POINTER(vp_amg_opts)]),
        "vp_amg_apply": (I, [P, P, P]),
        "vp_amg_info": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
        "vp_amg_export": (I, [P, I, P, P]),
        "vp_amg_rs_info": (I, [P, I, P]),
        "vp_amg_rs_export": (I, [P, I, P, P, P, P, P, P, P, P]),
        "vp_krylov_solve": (I, [P, P, P, C.POINTER(vp_krylov_opts), C.POINTER(vp_krylov_info)]),
        "vp_krylov_solve_noalloc": (I, [P, P, P, C.POINTER(vp_krylov_opts), C.POINTER(vp_krylov_info)]),
        "vp_pi_update": (I, [P, P, P, P, D]),
        "vp_pi_init": (I, [P, P, P]),
        "vp_newton_step": (I, [P, P, P, C.POINTER(vp_newton_opts), C.POINTER(vp_amg_opts),
                               C.POINTER(vp_krylov_opts), C.POINTER(vp_newton_info)]),
        "vp_newton_solve": (I, [P, P, P, I, C.POINTER(vp_newton_opts), C.POINTER(vp_amg_opts),
                                C.POINTER(vp_krylov_opts), C.POINTER(vp_solve_info), P]),
        "vp_advect": (I, [P, P, P, P, P, P]),
        "vp_profile": (I, [P, I]),
        "vp_profile_read": (I, [P, I, C.POINTER(D), C.POINTER(I), C.POINTER(D)]),
        "vp_default_opts": (None, [C.POINTER(vp_newton_opts), C.POINTER(vp_amg_opts),
                                   C.POINTER(vp_krylov_opts)]),
        "vpnet_create": (I, [I, I, I, P, C.POINTER(P)]),
        "vpnet_destroy": (None, [P]),
        "vpnet_last_error": (C.c_char_p, [P]),
        "vpnet_param_count": (C.c_int64, [P]),
        "vpnet_set_params": (I, [P, P]),
        "vpnet_get_params": (I, [P, P]),
        "vpnet_get_grads": (I, [P, P]),
        "vpnet_forward": (I, [P, P, P]),
        "vpnet_backward": (I, [P, P, P, C.POINTER(C.c_float)]),
        "vpnet_adam": (I, [P, C.c_float]),
        "vpnet_train_step": (I, [P, P, P, C.c_float, C.POINTER(C.c_float)]),
        "vpnet_features": (I, [I, I, I, P, P, P, P, P, P, P]),
        "vpnet_targets": (I, [I, I, P, P, P, P, P]),
        "vpnet_guess": (I, [I, I, P, I, I, P, P, P, P]),
        "vpnet_infer": (I, [P, P, I, P, P, C.POINTER(I)]),
        "vpnet_inspect": (I, [P, I, P, P, C.POINTER(C.c_int64)]),
        "vpnet_gemm": (I, [P, P, P, I, I, I, I, I, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


class VPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvp error {code}: {msg}")
        self.code = code


def default_opts():
    n, a, k = vp_newton_opts(), vp_amg_opts(), vp_krylov_opts()
    LIB.vp_default_opts(C.byref(n), C.byref(a), C.byref(k))
    return n, a, k


def _ptr(t, shape, name, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() != int(torch.Size(shape).numel()):
        raise ValueError(f"{name}: expected {tuple(shape)} elements, got shape {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def desc_from(d) -> vp_problem_desc:
    return vp_problem_desc(d.nx, d.ny, d.Lx, d.Ly, d.rho_ice, d.rho_air, d.rho_ocean, d.C_air,
                           d.C_ocean, d.P_star, d.C_strength, d.e_ratio, d.f_coriolis, d.dt,
                           d.delta_min, int(getattr(d, "order", 1)))


class Context:
    """One libvp context bound to the current torch stream of the current device."""

    def __init__(self, desc, stream=None):
        self.desc = desc
        self.nx, self.ny = desc.nx, desc.ny
        self.order = int(getattr(desc, "order", 1))
        o = self.order
        self.node_shape = ((o * desc.ny + 1) * (o * desc.nx + 1), 2)
        self.cell_shape = (desc.ny, desc.nx)
        self.pi_shape = (4 if o == 1 else 9, 3, desc.ny, desc.nx)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        self._d = desc_from(desc)
        rc = LIB.vp_create(C.byref(self._d), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise VPError(rc, LIB.vp_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            LIB.vp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, soft_ok=True):
        if rc < 0 or (rc > 0 and not soft_ok):
            raise VPError(rc, LIB.vp_last_error(self.h).decode())
        return rc

    # --- the C ABI, one method per entry point --------------------------------------
    def vp_set_state(self, H, A, v_air, v_ocean, v_prev):
        return self._check(LIB.vp_set_state(
            self.h, _ptr(H, self.cell_shape, "H"), _ptr(A, self.cell_shape, "A"),
            _ptr(v_air, self.node_shape, "v_air"), _ptr(v_ocean, self.node_shape, "v_ocean"),
            _ptr(v_prev, self.node_shape, "v_prev")))

    def vp_residual(self, v, r=None, want_scalars=True):
        rn, en = C.c_double(), C.c_double()
        rc = LIB.vp_residual(self.h, _ptr(v, self.node_shape, "v"), _ptr(r, self.node_shape, "r"),
                             C.byref(rn) if want_scalars else None,
                             C.byref(en) if want_scalars else None)
        self._check(rc)
        return (rn.value, en.value) if want_scalars else None

    def vp_newton_assemble(self, v, pi, variant=VP_SVN):
        return self._check(LIB.vp_newton_assemble(
            self.h, _ptr(v, self.node_shape, "v"),
            _ptr(pi, self.pi_shape, "pi") if pi is not None else None, variant))

    def vp_operator_apply(self, x, y):
        return self._check(LIB.vp_operator_apply(self.h, _ptr(x, self.node_shape, "x"),
                                                 _ptr(y, self.node_shape, "y")))

    def vp_operator_export(self, blocks):
        """blocks: [5 or 13 stored blocks x 4 values, nodes] (Q1 / Q2), layout [blk][node][r][c]."""
        n = self.node_shape[0]
        nb = 20 if self.order == 1 else 52
        return self._check(LIB.vp_operator_export(self.h, _ptr(blocks, (nb, n), "blocks")))

    def vp_amg_setup(self, opts=None):
        if opts is None:
            opts = default_opts()[1]
        return self._check(LIB.vp_amg_setup(self.h, C.byref(opts)))

    def vp_amg_apply(self, r, z):
        return self._check(LIB.vp_amg_apply(self.h, _ptr(r, self.node_shape, "r"),
                                            _ptr(z, self.node_shape, "z")))

    def vp_amg_info(self):
        lv = C.c_int()
        nx = (C.c_int * 32)()
        ny = (C.c_int * 32)()
        b = (C.c_int * 32)()
        self._check(LIB.vp_amg_info(self.h, C.byref(lv), nx, ny, b))
        return [(nx[i], ny[i], b[i]) for i in range(lv.value)]

    def vp_amg_export(self, level, A=None, P=None):
        """A: [5*B*B, nn] (layout of vp_operator_export, B x B blocks); P: [12*B, nn]."""
        lv = self.vp_amg_info()
        if not 0 <= level < len(lv):
            raise ValueError("level out of range")
        nxn, nyn, B = lv[level]
        nn = nxn * nyn
        pa = _ptr(A, (5 * B * B * nn,), "A") if A is not None else None
        pp = _ptr(P, (12 * B * nn,), "P") if P is not None else None
        return self._check(LIB.vp_amg_export(self.h, int(level), pa, pp))

    def vp_amg_rs_info(self, level):
        """Classical AMG level sizes: (rows, entries of A, coarse points, entries of P, colours)."""
        out = (C.c_int64 * 5)()
        self._check(LIB.vp_amg_rs_info(self.h, int(level), out))
        return tuple(int(v) for v in out)

    def vp_amg_rs_export(self, level):
        """Classical AMG level `level` as device tensors: dict with A (ptr, col, val),
        and below the coarsest level cf, P (ptr, col, val) and colour."""
        n, nnz, nc, nnzp, ncol = self.vp_amg_rs_info(level)
        dev = torch.device("cuda")
        i32 = torch.int32
        out = dict(n=n, nc=nc, ncol=ncol,
                   A_ptr=torch.empty(n + 1, dtype=i32, device=dev), A_col=torch.empty(max(nnz, 1), dtype=i32, device=dev),
                   A_val=torch.empty(max(nnz, 1), dtype=torch.float64, device=dev))
        args = [_ptr(out["A_ptr"], (n + 1,), "A_ptr", i32), _ptr(out["A_col"], out["A_col"].shape, "A_col", i32),
                _ptr(out["A_val"], out["A_val"].shape, "A_val")]
        if nc > 0:
            out.update(cf=torch.empty(n, dtype=i32, device=dev), P_ptr=torch.empty(n + 1, dtype=i32, device=dev),
                       P_col=torch.empty(max(nnzp, 1), dtype=i32, device=dev),
                       P_val=torch.empty(max(nnzp, 1), dtype=torch.float64, device=dev),
                       colour=torch.empty(n, dtype=i32, device=dev))
            args += [_ptr(out["cf"], (n,), "cf", i32), _ptr(out["P_ptr"], (n + 1,), "P_ptr", i32),
                     _ptr(out["P_col"], out["P_col"].shape, "P_col", i32), _ptr(out["P_val"], out["P_val"].shape, "P_val"),
                     _ptr(out["colour"], (n,), "colour", i32)]
        else:
            args += [None] * 5
        self._check(LIB.vp_amg_rs_export(self.h, int(level), *args))
        torch.cuda.synchronize()
        out["A_col"], out["A_val"] = out["A_col"][:nnz], out["A_val"][:nnz]
        if nc > 0:
            out["P_col"], out["P_val"] = out["P_col"][:nnzp], out["P_val"][:nnzp]
        return out

    def vp_krylov_solve(self, b, x, opts=None):
        if opts is None:
            opts = default_opts()[2]
        info = vp_krylov_info()
        rc = self._check(LIB.vp_krylov_solve(self.h, _ptr(b, self.node_shape, "b"),
                                             _ptr(x, self.node_shape, "x"), C.byref(opts),
                                             C.byref(info)))
        return rc, info

    def vp_krylov_solve_noalloc(self, b, x, opts=None):
        if opts is None:
            opts = default_opts()[2]
        info = vp_krylov_info()
        rc = self._check(LIB.vp_krylov_solve_noalloc(self.h, _ptr(b, self.node_shape, "b"),
                                                     _ptr(x, self.node_shape, "x"), C.byref(opts),
                                                     C.byref(info)))
        return rc, info

    def vp_pi_update(self, v, dv, pi, alpha):
        return self._check(LIB.vp_pi_update(self.h, _ptr(v, self.node_shape, "v"),
                                            _ptr(dv, self.node_shape, "dv"),
                                            _ptr(pi, self.pi_shape, "pi"), float(alpha)))

    def vp_pi_init(self, v, pi):
        return self._check(LIB.vp_pi_init(self.h, _ptr(v, self.node_shape, "v"),
                                          _ptr(pi, self.pi_shape, "pi")))

    def vp_newton_step(self, v, pi, nopts=None, aopts=None, kopts=None):
        dn, da, dk = default_opts()
        info = vp_newton_info()
        rc = self._check(LIB.vp_newton_step(
            self.h, _ptr(v, self.node_shape, "v"),
            _ptr(pi, self.pi_shape, "pi") if pi is not None else None,
            C.byref(nopts or dn), C.byref(aopts or da), C.byref(kopts or dk), C.byref(info)))
        return rc, info

    def vp_advect(self, v, A, H, A_out, H_out):
        return self._check(LIB.vp_advect(
            self.h, _ptr(v, self.node_shape, "v"), _ptr(A, self.cell_shape, "A"), _ptr(H, self.cell_shape, "H"),
            _ptr(A_out, self.cell_shape, "A_out"), _ptr(H_out, self.cell_shape, "H_out")))

    def vp_profile(self, enable):
        return self._check(LIB.vp_profile(self.h, int(bool(enable))))

    def vp_profile_read(self, kid):
        ms, n, b = C.c_double(), C.c_int(), C.c_double()
        self._check(LIB.vp_profile_read(self.h, int(kid), C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def vp_newton_solve(self, v, pi, maxit=200, nopts=None, aopts=None, kopts=None, history=True):
        dn, da, dk = default_opts()
        info = vp_solve_info()
        hist = (C.c_double * (maxit + 1))() if history else None
        rc = self._check(LIB.vp_newton_solve(
            self.h, _ptr(v, self.node_shape, "v"),
            _ptr(pi, self.pi_shape, "pi") if pi is not None else None, int(maxit),
            C.byref(nopts or dn), C.byref(aopts or da), C.byref(kopts or dk), C.byref(info),
            hist))
        h = list(hist[: info.iterations + 1]) if history else None
        return rc, info, h


def to_device(arr, device="cuda"):
    return torch.as_tensor(arr, dtype=torch.float64).contiguous().to(device)


def context_for(workload, device="cuda"):
    """Create a context for a seeded workload and upload its state."""
    ctx = Context(workload.desc)
    f = workload.fields()
    ts = {k: to_device(v.reshape(-1, 2) if v.ndim == 3 else v, device) for k, v in f.items()}
    ctx.vp_set_state(ts["H"], ts["A"], ts["v_air"], ts["v_ocean"], ts["v_prev"])
    ctx._state = ts
    return ctx


# ---------------------------------------------------------------------------
# learned warm start (include/vpnet.h)
# ---------------------------------------------------------------------------
def _fptr(t, numel, name, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous CUDA {dtype} tensor")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    """One U-Net instance for a fixed batch and spatial size (NHWC tensors)."""

    def __init__(self, batch, height, width):
        self.B, self.H, self.W = batch, height, width
        h = C.c_void_p()
        rc = LIB.vpnet_create(batch, height, width, _stream(), C.byref(h))
        if rc != 0:
            raise VPError(rc, "vpnet_create failed (batch >= 1, H and W multiples of 8)")
        self.h = h
        self.nparam = int(LIB.vpnet_param_count(h))

    def close(self):
        if getattr(self, "h", None):
            LIB.vpnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise VPError(rc, LIB.vpnet_last_error(self.h).decode())
        return rc

    def vpnet_set_params(self, theta):
        return self._check(LIB.vpnet_set_params(self.h, _fptr(theta, self.nparam, "theta")))

    def vpnet_get_params(self, out):
        return self._check(LIB.vpnet_get_params(self.h, _fptr(out, self.nparam, "out")))

    def vpnet_get_grads(self, out):
        return self._check(LIB.vpnet_get_grads(self.h, _fptr(out, self.nparam, "out")))

    def vpnet_forward(self, x, out):
        P = self.B * self.H * self.W
        return self._check(LIB.vpnet_forward(self.h, _fptr(x, P * 8, "x"), _fptr(out, P * 5, "out")))

    def vpnet_backward(self, x, target):
        P = self.B * self.H * self.W
        loss = C.c_float()
        self._check(LIB.vpnet_backward(self.h, _fptr(x, P * 8, "x"), _fptr(target, P * 5, "target"),
                                       C.byref(loss)))
        return loss.value

    def vpnet_adam(self, lr):
        return self._check(LIB.vpnet_adam(self.h, C.c_float(lr)))

    def vpnet_infer(self, ctx, candidates, v0, pi0):
        """Learned start for ctx's current state, chosen by energy among `candidates`
        (names from START); returns the chosen name."""
        mask = 0
        for c in candidates:
            mask |= START[c]
        chosen = C.c_int()
        self._check(LIB.vpnet_infer(self.h, ctx.h, mask, _ptr(v0, ctx.node_shape, "v0"),
                                    _ptr(pi0, ctx.pi_shape, "pi0"), C.byref(chosen)))
        return {v: k for k, v in START.items()}[chosen.value]

    def vpnet_inspect(self, act, want_grad=True):
        """(values, gradient) of activation `act` as flat CUDA float32 tensors."""
        cnt = C.c_int64()
        self._check(LIB.vpnet_inspect(self.h, int(act), None, None, C.byref(cnt)))
        y = torch.empty(cnt.value, dtype=torch.float32, device="cuda")
        g = torch.empty_like(y) if want_grad else None
        self._check(LIB.vpnet_inspect(self.h, int(act), C.c_void_p(y.data_ptr()),
                                      C.c_void_p(g.data_ptr()) if g is not None else None, None))
        return y, g

    def vpnet_train_step(self, x, target, lr, want_loss=True):
        P = self.B * self.H * self.W
        loss = C.c_float()
        self._check(LIB.vpnet_train_step(self.h, _fptr(x, P * 8, "x"), _fptr(target, P * 5, "target"),
                                         C.c_float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def vpnet_features(nx, ny, f, H, A, v_air, v_ocean, v_prev, out):
    nn = (nx + 1) * (ny + 1)
    if nx % f or ny % f:
        raise ValueError("pool factor must divide the mesh")
    rc = LIB.vpnet_features(nx, ny, f, _fptr(H, nx * ny, "H", torch.float64),
                            _fptr(A, nx * ny, "A", torch.float64),
                            _fptr(v_air, 2 * nn, "v_air", torch.float64),
                            _fptr(v_ocean, 2 * nn, "v_ocean", torch.float64),
                            _fptr(v_prev, 2 * nn, "v_prev", torch.float64),
                            _fptr(out, (nx // f) * (ny // f) * 8, "out"), _stream())
    if rc != 0:
        raise VPError(rc, "vpnet_features")


def vpnet_targets(nx, ny, v, pi, out, v_prev=None):
    rc = LIB.vpnet_targets(nx, ny, _fptr(v, 2 * (nx + 1) * (ny + 1), "v", torch.float64),
                           _fptr(pi, 12 * nx * ny, "pi", torch.float64),
                           _fptr(v_prev, 2 * (nx + 1) * (ny + 1), "v_prev", torch.float64),
                           _fptr(out, nx * ny * 5, "out"), _stream())
    if rc != 0:
        raise VPError(rc, "vpnet_targets")


def vpnet_guess(nx, ny, net_out, wc, hc, v0, pi0, v_prev=None):
    rc = LIB.vpnet_guess(nx, ny, _fptr(net_out, wc * hc * 5, "net_out"), wc, hc,
                         _fptr(v_prev, 2 * (nx + 1) * (ny + 1), "v_prev", torch.float64),
                         _fptr(v0, 2 * (nx + 1) * (ny + 1), "v0", torch.float64),
                         _fptr(pi0, 12 * nx * ny, "pi0", torch.float64) if pi0 is not None else None,
                         _stream())
    if rc != 0:
        raise VPError(rc, "vpnet_guess")


def vpnet_gemm(A, B, C_out, M, N, K, a_trans=False, b_trans=False):
    for t, nme, n in ((A, "A", M * K), (B, "B", K * N)):
        if t.dtype != torch.bfloat16 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise TypeError(f"{nme}: expected a contiguous CUDA bfloat16 tensor of {n} elements")
    rc = LIB.vpnet_gemm(C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()),
                        _fptr(C_out, M * N, "C"), M, N, K, int(a_trans), int(b_trans), _stream())
    if rc != 0:
        raise VPError(rc, "vpnet_gemm")
