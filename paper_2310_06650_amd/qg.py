"""ctypes binding of the qg C ABI (include/qg.h).

The functions named like the C entry points only marshal arguments and raise
QgError on a non-OK status; every step of the hot path runs in the HIP library
libqg.so, which must be built (``python -m paper_2310_06650_amd.build``).
There is no fallback: importing this module without the library fails.

``Problem`` is a convenience owner of the device buffers (torch tensors) of one
problem.  PyTorch only provides device memory and streams here.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QG_LIBRARY names another build of the same library (the host-sanitized one
# of build.build(sanitize=True)); by default the in-tree libqg.so
LIB_PATH = os.environ.get("QG_LIBRARY") or os.path.join(_HERE, "libqg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2310_06650_amd.build)")
# PyTorch ships its own HIP runtime under the same soname as the system one.
# Importing it first makes the library bind to that runtime, so one process
# holds a single HIP runtime whichever module is imported first.
import torch as _torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
QG_OK, QG_ERR_ARG, QG_ERR_TOPOLOGY, QG_ERR_SINGULAR, QG_ERR_NONFINITE, \
    QG_ERR_DEVICE, QG_ERR_STATE = range(7)
TERM_NAMES = ("dev", "bal", "br", "ang", "pen", "rsv", "ctg_max", "ctg_mean",
              "load_value", "total")
QG_NTERMS = 10
QG_NCLASS = 6
QG_NKERNELS = 8
QG_CTG_ALL_NONBRIDGE, QG_CTG_LIST = 0, 1
QG_FLAG_CHECK_FINITE = 0x1
QG_FLAG_CTG_FP32 = 0x2
QG_FLAG_CTG_BF16 = 0x4
QG_FLAG_CTG_SUM = 0x8
QG_FLAG_CTG_NO_SKIP = 0x10
QG_NOALLOC_SCRATCH = 32 << 20   # bytes of qg_eval_grad_noalloc's static scratch

KERNEL_NAMES = ("k_forward", "k_ctg_main", "k_ctg_zred", "k_ctg_asm", "k_adjoint", "k_final")

_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int32)


class qg_grid_desc(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_branch", C.c_int32), ("n_gen", C.c_int32),
        ("n_period", C.c_int32), ("n_seg", C.c_int32),
        ("br_from", _pi), ("br_to", _pi),
        ("br_r", _pd), ("br_x", _pd), ("br_bch", _pd), ("br_smax", _pd), ("br_smax_ctg", _pd),
        ("gen_bus", _pi),
        ("gen_pmin", _pd), ("gen_pmax", _pd), ("gen_qmin", _pd), ("gen_qmax", _pd),
        ("gen_rmax", _pd), ("gen_ru", _pd), ("gen_rd", _pd), ("gen_ru_su", _pd),
        ("gen_rd_sd", _pd), ("gen_p0", _pd), ("gen_u0", _pd), ("gen_c_on", _pd),
        ("gen_c_su", _pd), ("gen_c_sd", _pd), ("gen_c_r", _pd),
        ("gen_seg_cost", _pd), ("gen_seg_size", _pd),
        ("load_p", _pd), ("load_q", _pd), ("reserve_req", _pd), ("dt", _pd),
        ("v_min", _pd), ("v_max", _pd),
        ("c_p", C.c_double), ("c_q", C.c_double), ("c_s", C.c_double),
        ("c_ang", C.c_double), ("ang_max", C.c_double), ("c_rsv", C.c_double),
        ("rho", C.c_double), ("load_value", C.c_double)]


class qg_build_opts(C.Structure):
    _fields_ = [("ref_bus", C.c_int32), ("ctg_mode", C.c_int32), ("ctg_list", _pi),
                ("n_ctg", C.c_int32), ("flags", C.c_uint32)]


class qg_sizes(C.Structure):
    _fields_ = [("const_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
                ("n_x", C.c_int64), ("n_ctg", C.c_int32)]


class qg_layout(C.Structure):
    _fields_ = [("off", C.c_int64 * QG_NCLASS), ("len", C.c_int64 * QG_NCLASS)]


class qg_homotopy(C.Structure):
    _fields_ = [("eps", C.c_double), ("beta", C.c_double), ("rho_scale", C.c_double)]


class qg_adam_cfg(C.Structure):
    _fields_ = [("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("eps_in_numerator", C.c_int32)]


class qg_solve_opts(C.Structure):
    _fields_ = [("n_steps", C.c_int64), ("iter0", C.c_int64), ("n_total", C.c_int64),
                ("check_every", C.c_int64),
                ("alpha0", C.c_double * QG_NCLASS), ("alphaf", C.c_double * QG_NCLASS),
                ("eps0", C.c_double), ("epsf", C.c_double), ("beta0", C.c_double),
                ("betaf", C.c_double), ("rho0", C.c_double), ("rhof", C.c_double),
                ("z_ed", C.c_double), ("stop_ratio", C.c_double),
                ("use_graph", C.c_int32), ("profile", C.c_int32),
                ("skip_final", C.c_int32), ("reserved", C.c_int32)]


class qg_solve_report(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("steps_to_gap", C.c_int64),
                ("wall_s", C.c_double), ("time_to_gap_s", C.c_double),
                ("final_loss", C.c_double), ("final_score", C.c_double),
                ("terms", C.c_double * QG_NTERMS),
                ("kernel_ms", C.c_double * QG_NKERNELS),
                ("kernel_calls", C.c_int64 * QG_NKERNELS),
                ("steps_ms", C.c_double)]


class qg_screen_opts(C.Structure):
    _fields_ = [("top_frac", C.c_double), ("rand_frac", C.c_double), ("zeta", C.c_double),
                ("refresh_every", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64)]


QG_MLP_MAX_DEPTH = 8


class qg_mlp_desc(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("d_out", C.c_int32)]


class qg_mlp_layout(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("w_off", C.c_int64 * (QG_MLP_MAX_DEPTH + 1)),
                ("b_off", C.c_int64 * (QG_MLP_MAX_DEPTH + 1))]


_vp = C.c_void_p
_sig = {
    "qg_problem_sizes": (C.c_int, [C.POINTER(qg_grid_desc), C.POINTER(qg_build_opts),
                                   C.POINTER(qg_sizes)]),
    "qg_build_problem": (C.c_int, [C.POINTER(qg_grid_desc), C.POINTER(qg_build_opts), _vp,
                                   C.c_size_t, _vp, C.POINTER(_vp)]),
    "qg_layout_of": (C.c_int, [_vp, C.POINTER(qg_layout)]),
    "qg_ctg_list": (C.c_int, [_vp, _pi, C.c_int32]),
    "qg_problem_dims": (C.c_int, [_vp, _pi, C.c_int32]),
    "qg_update_loads": (C.c_int, [_vp, _pd, _pd, _pd, _vp]),
    "qg_time_stage": (C.c_int, [_vp, _vp, C.POINTER(qg_homotopy), C.c_int32, C.c_int32, _vp,
                                _vp, C.POINTER(C.c_double)]),
    "qg_set_ctg_tile": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "qg_set_ctg_ltiles": (C.c_int, [_vp, C.c_int32]),
    "qg_set_ctg_tile_split": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
    "qg_eval_grad": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(qg_homotopy), _vp, _vp]),
    "qg_eval_grad_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(qg_homotopy), _vp]),
    "qg_adam_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int64, C.c_double * QG_NCLASS,
                               C.POINTER(qg_adam_cfg), _vp]),
    "qg_solve": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(qg_solve_opts),
                           C.POINTER(qg_adam_cfg), C.POINTER(qg_solve_report), _vp, _vp]),
    "qg_debug_fetch": (C.c_int, [_vp, _vp, C.c_char_p, _vp, C.c_size_t, _vp]),
    "qg_batch_bytes": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(C.c_size_t)]),
    "qg_build_image": (C.c_int, [C.POINTER(qg_grid_desc), C.POINTER(qg_build_opts), _vp,
                                 C.c_size_t]),
    "qg_solve_batch": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(_vp), C.POINTER(_vp),
                                 C.POINTER(_vp), C.POINTER(_vp), _vp, C.c_size_t,
                                 C.POINTER(qg_solve_opts), C.POINTER(qg_adam_cfg),
                                 C.POINTER(qg_solve_report), _vp]),
    "qg_screen_bytes": (C.c_int, [_vp, C.POINTER(qg_screen_opts), C.POINTER(C.c_size_t)]),
    "qg_set_screening": (C.c_int, [_vp, C.POINTER(qg_screen_opts), _vp, C.c_size_t, _vp]),
    "qg_screen_refresh": (C.c_int, [_vp, _vp, C.POINTER(qg_homotopy), C.c_int64, _vp, _vp]),
    "qg_set_active_contingencies": (C.c_int, [_vp, _pi, C.c_int32, _vp]),
    "qg_get_active_contingencies": (C.c_int, [_vp, _pi, C.c_int32, _pi, _pd, _vp]),
    "qg_destroy_problem": (None, [_vp]),
    "qg_mlp_sizes": (C.c_int, [C.POINTER(qg_mlp_desc), C.c_int32, C.POINTER(qg_mlp_layout),
                               C.POINTER(C.c_size_t)]),
    "qg_mlp_forward": (C.c_int, [C.POINTER(qg_mlp_desc), _vp, _vp, C.c_int32, _vp, _vp, _vp]),
    "qg_mlp_grad": (C.c_int, [C.POINTER(qg_mlp_desc), _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp,
                              _vp]),
    "qg_mlp_train_step": (C.c_int, [C.POINTER(qg_mlp_desc), _vp, _vp, _vp, _vp, _vp, _vp,
                                    C.c_int32, C.c_int64, C.c_float, _vp, _vp, _vp]),
    "qg_mlp_to_bf16": (C.c_int, [C.POINTER(qg_mlp_desc), _vp, _vp, _vp]),
    "qg_mlp_forward_bf16": (C.c_int, [C.POINTER(qg_mlp_desc), _vp, _vp, C.c_int32, _vp, _vp,
                                      _vp]),
    "qg_status_string": (C.c_char_p, [C.c_int]),
    "qg_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class QgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = lib.qg_last_error().decode()
        super().__init__(f"{where}: {lib.qg_status_string(status).decode()} ({status}): {detail}")


def _check(status, where):
    if status != QG_OK:
        raise QgError(status, where)


# ---------------------------------------------------------------- marshalling

def grid_desc(case):
    """qg_grid_desc for a GridCase; returns (desc, keepalive)."""
    keep = []

    def d(a):
        arr = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(arr)
        return arr.ctypes.data_as(_pd)

    def i(a):
        arr = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(arr)
        return arr.ctypes.data_as(_pi)

    c = case
    desc = qg_grid_desc(
        n_bus=c.n_bus, n_branch=c.n_branch, n_gen=c.n_gen, n_period=c.n_period,
        n_seg=c.n_seg, br_from=i(c.br_from), br_to=i(c.br_to), br_r=d(c.br_r),
        br_x=d(c.br_x), br_bch=d(c.br_bch), br_smax=d(c.br_smax),
        br_smax_ctg=d(c.br_smax_ctg), gen_bus=i(c.gen_bus), gen_pmin=d(c.gen_pmin),
        gen_pmax=d(c.gen_pmax), gen_qmin=d(c.gen_qmin), gen_qmax=d(c.gen_qmax),
        gen_rmax=d(c.gen_rmax), gen_ru=d(c.gen_ru), gen_rd=d(c.gen_rd),
        gen_ru_su=d(c.gen_ru_su), gen_rd_sd=d(c.gen_rd_sd), gen_p0=d(c.gen_p0),
        gen_u0=d(c.gen_u0), gen_c_on=d(c.gen_c_on), gen_c_su=d(c.gen_c_su),
        gen_c_sd=d(c.gen_c_sd), gen_c_r=d(c.gen_c_r), gen_seg_cost=d(c.gen_seg_cost),
        gen_seg_size=d(c.gen_seg_size), load_p=d(c.load_p), load_q=d(c.load_q),
        reserve_req=d(c.reserve_req), dt=d(c.dt), v_min=d(c.v_min), v_max=d(c.v_max),
        c_p=c.c_p, c_q=c.c_q, c_s=c.c_s, c_ang=c.c_ang, ang_max=c.ang_max,
        c_rsv=c.c_rsv, rho=c.rho, load_value=c.load_value)
    return desc, keep


def build_opts(case=None, ctg_mode=QG_CTG_LIST, ctg_list=None, ref_bus=None, flags=0):
    keep = []
    if ctg_list is None and case is not None and ctg_mode == QG_CTG_LIST:
        ctg_list = case.ctg_list
    ptr = None
    n = 0
    if ctg_list is not None:
        arr = np.ascontiguousarray(ctg_list, dtype=np.int32)
        keep.append(arr)
        ptr = arr.ctypes.data_as(_pi)
        n = int(arr.shape[0])
    if ref_bus is None:
        ref_bus = case.ref_bus if case is not None else 0
    return qg_build_opts(ref_bus=ref_bus, ctg_mode=ctg_mode, ctg_list=ptr, n_ctg=n,
                         flags=flags), keep


# ---------------------------------------------------------------- C-named calls

def qg_problem_sizes(desc, opts):
    out = qg_sizes()
    _check(lib.qg_problem_sizes(C.byref(desc), C.byref(opts), C.byref(out)), "qg_problem_sizes")
    return out


def qg_build_image(desc, opts, nbytes):
    """The constant arena's image, built on the host (numpy uint8 array)."""
    out = np.zeros(max(int(nbytes), 1), dtype=np.uint8)
    _check(lib.qg_build_image(C.byref(desc), C.byref(opts), out.ctypes.data_as(_vp),
                              out.nbytes), "qg_build_image")
    return out


def qg_build_problem(desc, opts, d_arena, const_bytes, stream):
    h = _vp()
    _check(lib.qg_build_problem(C.byref(desc), C.byref(opts), d_arena, const_bytes, stream,
                                C.byref(h)), "qg_build_problem")
    return h


def qg_layout_of(h):
    out = qg_layout()
    _check(lib.qg_layout_of(h, C.byref(out)), "qg_layout_of")
    return out


def qg_ctg_list(h, k):
    out = np.zeros(max(k, 1), dtype=np.int32)
    _check(lib.qg_ctg_list(h, out.ctypes.data_as(_pi), out.shape[0]), "qg_ctg_list")
    return out[:k]


def qg_problem_dims(h):
    out = np.zeros(19, dtype=np.int32)
    _check(lib.qg_problem_dims(h, out.ctypes.data_as(_pi), 19), "qg_problem_dims")
    keys = ("N", "L", "G", "T", "M", "K", "Lp", "Kp", "G16", "G4", "Tp", "nLb", "nKb",
            "ctg_bl", "ctg_wl", "ctg_tc", "lodf_kind", "ctg_lt", "ctg_split")
    return dict(zip(keys, (int(v) for v in out)))


def qg_set_ctg_tile(h, bl, wl, tc=0):
    _check(lib.qg_set_ctg_tile(h, bl, wl, tc), "qg_set_ctg_tile")


def qg_eval_grad(h, d_x, d_grad, d_terms, hom, d_ws, stream):
    _check(lib.qg_eval_grad(h, d_x, d_grad, d_terms, C.byref(hom), d_ws, stream),
           "qg_eval_grad")


def qg_eval_grad_noalloc(h, d_x, d_grad, d_terms, hom, stream):
    _check(lib.qg_eval_grad_noalloc(h, d_x, d_grad, d_terms, C.byref(hom), stream),
           "qg_eval_grad_noalloc")


def qg_time_stage(h, d_x, hom, stage, reps, d_ws, stream):
    out = C.c_double(0.0)
    _check(lib.qg_time_stage(h, d_x, C.byref(hom), int(stage), int(reps), d_ws, stream,
                             C.byref(out)), "qg_time_stage")
    return out.value


def qg_adam_step(h, d_x, d_m, d_v, d_g, it, lr, cfg, stream):
    arr = (C.c_double * QG_NCLASS)(*[float(a) for a in lr])
    _check(lib.qg_adam_step(h, d_x, d_m, d_v, d_g, int(it), arr, C.byref(cfg), stream),
           "qg_adam_step")


def qg_solve(h, d_x, d_m, d_v, opts, cfg, d_ws, stream):
    rep = qg_solve_report()
    _check(lib.qg_solve(h, d_x, d_m, d_v, C.byref(opts), C.byref(cfg), C.byref(rep), d_ws,
                        stream), "qg_solve")
    return rep


def qg_debug_fetch(h, d_ws, name, host_array, stream):
    _check(lib.qg_debug_fetch(h, d_ws, name.encode(), host_array.ctypes.data_as(_vp),
                              host_array.nbytes, stream), "qg_debug_fetch")
    return host_array


def qg_destroy_problem(h):
    lib.qg_destroy_problem(h)


# ---------------------------------------------------------------- owner class

def solve_opts(n_steps, alpha0, alphaf=None, iter0=0, n_total=0, check_every=0, eps0=1e-2,
               epsf=1e-2, beta0=1.0, betaf=1.0, rho0=1.0, rhof=1.0, z_ed=0.0,
               stop_ratio=0.99, use_graph=1, profile=0, skip_final=0):
    alpha0 = list(alpha0) if np.ndim(alpha0) else [float(alpha0)] * QG_NCLASS
    alphaf = alpha0 if alphaf is None else (
        list(alphaf) if np.ndim(alphaf) else [float(alphaf)] * QG_NCLASS)
    return qg_solve_opts(
        n_steps=n_steps, iter0=iter0, n_total=n_total, check_every=check_every,
        alpha0=(C.c_double * QG_NCLASS)(*alpha0), alphaf=(C.c_double * QG_NCLASS)(*alphaf),
        eps0=eps0, epsf=epsf, beta0=beta0, betaf=betaf, rho0=rho0, rhof=rhof, z_ed=z_ed,
        stop_ratio=stop_ratio, use_graph=use_graph, profile=profile,
        skip_final=1 if skip_final else 0, reserved=0)


def adam_cfg(beta1=0.9, beta2=0.999, eps=1e-8, eps_in_numerator=False):
    return qg_adam_cfg(beta1=beta1, beta2=beta2, eps=eps,
                       eps_in_numerator=1 if eps_in_numerator else 0)


class Problem:
    """Device buffers and handle of one built problem (torch tensors on a GPU)."""

    def __init__(self, case, device="cuda", ctg_mode=QG_CTG_LIST, ctg_list=None, flags=0,
                 stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.case = case
        desc, keep1 = grid_desc(case)
        opts, keep2 = build_opts(case, ctg_mode=ctg_mode, ctg_list=ctg_list, flags=flags)
        self.sizes = qg_problem_sizes(desc, opts)
        self.arena = torch.empty(max(self.sizes.const_bytes, 256), dtype=torch.uint8,
                                 device=self.device)
        self.workspace = torch.empty(max(self.sizes.workspace_bytes, 256), dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream
        self.handle = qg_build_problem(desc, opts, self.arena.data_ptr(),
                                       self.sizes.const_bytes, self._stream())
        del keep1, keep2
        self.n_x = int(self.sizes.n_x)
        self.dims = qg_problem_dims(self.handle)
        self.K = self.dims["K"]

    def _stream(self):
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def layout(self):
        lay = qg_layout_of(self.handle)
        return list(lay.off), list(lay.len)

    def ctg_list(self):
        return qg_ctg_list(self.handle, self.K)

    def set_ctg_tile(self, bl, wl, tc=0, lt=None):
        qg_set_ctg_tile(self.handle, bl, wl, tc)
        if lt is not None:
            _check(lib.qg_set_ctg_ltiles(self.handle, int(lt)), "qg_set_ctg_ltiles")
        self.dims = qg_problem_dims(self.handle)

    def set_ctg_ltiles(self, lt):
        _check(lib.qg_set_ctg_ltiles(self.handle, int(lt)), "qg_set_ctg_ltiles")
        self.dims = qg_problem_dims(self.handle)

    def set_ctg_tile_split(self, wl, tcw, lt=0):
        _check(lib.qg_set_ctg_tile_split(self.handle, int(wl), int(tcw), int(lt)),
               "qg_set_ctg_tile_split")
        self.dims = qg_problem_dims(self.handle)

    def tile(self):
        """The map-reduce tile as text: "s{wl}x{tcw}x{lt}" for a period-split
        tile, "{bl}x{wl}x{tc}x{lt}" for a branch-stacked one."""
        d = self.dims
        if d["ctg_split"]:
            return f"s{d['ctg_wl']}x{d['ctg_tc']}x{d['ctg_lt']}"
        return f"{d['ctg_bl']}x{d['ctg_wl']}x{d['ctg_tc']}x{d['ctg_lt']}"

    def set_tile(self, text):
        """Set a tile given in the text form of tile(); lt may be left out or
        0 (the default)."""
        if text.startswith("s"):
            v = [int(u) for u in text[1:].split("x")]
            self.set_ctg_tile_split(v[0], v[1], v[2] if len(v) > 2 else 0)
        else:
            v = [int(u) for u in text.split("x")]
            self.set_ctg_tile(v[0], v[1], v[2], lt=(v[3] if len(v) > 3 else None))

    def new_vector(self, host=None):
        t = self.torch.zeros(self.n_x, dtype=self.torch.float64, device=self.device)
        if host is not None:
            t.copy_(self.torch.as_tensor(np.asarray(host, dtype=np.float64)))
        return t

    def update_loads(self, load_p, load_q, reserve_req):
        """Same grid, new loads (arrays [T, N], [T, N], [T])."""
        lp = np.ascontiguousarray(load_p, dtype=np.float64).reshape(-1)
        lq = np.ascontiguousarray(load_q, dtype=np.float64).reshape(-1)
        rr = np.ascontiguousarray(reserve_req, dtype=np.float64).reshape(-1)
        if lp.size != self.dims["T"] * self.dims["N"] or lq.size != lp.size or \
                rr.size != self.dims["T"]:
            raise ValueError("load arrays do not match the grid")
        _check(lib.qg_update_loads(self.handle, lp.ctypes.data_as(_pd), lq.ctypes.data_as(_pd),
                                   rr.ctypes.data_as(_pd), self._stream()), "qg_update_loads")

    def time_stage(self, x, stage, reps, eps, beta=1.0, rho_scale=1.0):
        """Mean microseconds of one kernel of the step (index into KERNEL_NAMES)."""
        if isinstance(stage, str):
            stage = KERNEL_NAMES.index(stage)
        return qg_time_stage(self.handle, x.data_ptr(), qg_homotopy(eps, beta, rho_scale), stage,
                             reps, self.workspace.data_ptr(), self._stream())

    def eval_grad(self, x, eps, beta=1.0, rho_scale=1.0, grad=True):
        torch = self.torch
        g = torch.empty(self.n_x, dtype=torch.float64, device=self.device) if grad else None
        terms = torch.empty(32, dtype=torch.float64, device=self.device)  # 256 B aligned
        qg_eval_grad(self.handle, x.data_ptr(), g.data_ptr() if g is not None else None,
                     terms.data_ptr(), qg_homotopy(eps, beta, rho_scale),
                     self.workspace.data_ptr(), self._stream())
        return terms[:QG_NTERMS], g

    def eval_grad_noalloc(self, x, eps, beta=1.0, rho_scale=1.0, grad=None, terms=None):
        """qg_eval_grad_noalloc into caller-given outputs (device tensors:
        grad [n_x] FP64 or None, terms of at least QG_NTERMS FP64 or None);
        the library's static scratch replaces the workspace."""
        qg_eval_grad_noalloc(self.handle, x.data_ptr(),
                             grad.data_ptr() if grad is not None else None,
                             terms.data_ptr() if terms is not None else None,
                             qg_homotopy(eps, beta, rho_scale), self._stream())
        return terms, grad

    def adam_step(self, x, m, v, g, it, lr, cfg=None):
        cfg = cfg or adam_cfg()
        lr = list(lr) if np.ndim(lr) else [float(lr)] * QG_NCLASS
        qg_adam_step(self.handle, x.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(), it,
                     lr, cfg, self._stream())

    def solve(self, x, m, v, opts, cfg=None):
        cfg = cfg or adam_cfg()
        return qg_solve(self.handle, x.data_ptr(), m.data_ptr(), v.data_ptr(), opts, cfg,
                        self.workspace.data_ptr(), self._stream())

    # ---- contingency screening (Alg. 2)

    def set_screening(self, top_frac=None, rand_frac=0.0, zeta=0.0, refresh=10, seed=0):
        """Screen contingencies (top_frac None: back to scoring all of them)."""
        if top_frac is None:
            _check(lib.qg_set_screening(self.handle, None, None, 0, self._stream()),
                   "qg_set_screening")
            self.screen_buf = None
            return
        o = qg_screen_opts(top_frac=top_frac, rand_frac=rand_frac, zeta=zeta,
                           refresh_every=refresh, reserved=0, seed=seed)
        nb = C.c_size_t(0)
        _check(lib.qg_screen_bytes(self.handle, C.byref(o), C.byref(nb)), "qg_screen_bytes")
        buf = self.torch.empty(max(nb.value, 256), dtype=self.torch.uint8, device=self.device)
        _check(lib.qg_set_screening(self.handle, C.byref(o), buf.data_ptr(), nb.value,
                                    self._stream()), "qg_set_screening")
        self.screen_buf = buf   # the library uses it until screening is reconfigured

    def screen_refresh(self, x, eps, beta=1.0, rho_scale=1.0, round=0):
        _check(lib.qg_screen_refresh(self.handle, x.data_ptr(), C.byref(qg_homotopy(
            eps, beta, rho_scale)), int(round), self.workspace.data_ptr(), self._stream()),
            "qg_screen_refresh")

    def set_active_contingencies(self, ks):
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        _check(lib.qg_set_active_contingencies(self.handle, ks.ctypes.data_as(_pi), ks.size,
                                               self._stream()), "qg_set_active_contingencies")

    def active_contingencies(self, severities=False):
        """The current set (and the severities of the last refresh)."""
        out = np.zeros(max(self.K, 1), dtype=np.int32)
        n = C.c_int32(0)
        sev = np.zeros(max(self.K, 1), dtype=np.float64) if severities else None
        _check(lib.qg_get_active_contingencies(
            self.handle, out.ctypes.data_as(_pi), out.size, C.byref(n),
            sev.ctypes.data_as(_pd) if sev is not None else None, self._stream()),
            "qg_get_active_contingencies")
        ks = out[:n.value].astype(np.int64)
        return (ks, sev[:self.K]) if severities else ks

    def fetch(self, name, shape):
        out = np.empty(shape, dtype=np.float64)
        return qg_debug_fetch(self.handle, self.workspace.data_ptr(), name, out, self._stream())

    def close(self):
        if getattr(self, "handle", None):
            qg_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def report_dict(rep):
    return dict(steps_done=rep.steps_done, steps_to_gap=rep.steps_to_gap, wall_s=rep.wall_s,
                time_to_gap_s=rep.time_to_gap_s, final_loss=rep.final_loss,
                final_score=rep.final_score,
                terms=dict(zip(TERM_NAMES, list(rep.terms))),
                kernel_ms=dict(zip(KERNEL_NAMES, list(rep.kernel_ms)[:len(KERNEL_NAMES)])),
                kernel_calls=dict(zip(KERNEL_NAMES, list(rep.kernel_calls)[:len(KERNEL_NAMES)])),
                steps_ms=rep.steps_ms)


class MLP:
    """Device buffers of the warm-start network (FP32 parameters, Adam moments,
    gradient scratch and workspace) on a GPU, driven through the qg_mlp ABI."""

    def __init__(self, d_in, width, depth, d_out, max_batch, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.desc = qg_mlp_desc(d_in, width, depth, d_out)
        self.layout = qg_mlp_layout()
        ws = C.c_size_t(0)
        _check(lib.qg_mlp_sizes(C.byref(self.desc), int(max_batch), C.byref(self.layout),
                                C.byref(ws)), "qg_mlp_sizes")
        self.max_batch = int(max_batch)
        self.n_params = int(self.layout.n_params)
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.zeros(self.n_params, **f32)
        self.m = torch.zeros(self.n_params, **f32)
        self.v = torch.zeros(self.n_params, **f32)
        self.grad = torch.zeros(self.n_params, **f32)
        self.loss = torch.zeros(64, **f32)
        self.workspace = torch.empty(int(ws.value) + 256, dtype=torch.uint8, device=self.device)
        self.params16 = None
        self.stream = stream
        self.iter = 0

    def _stream(self):
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def offsets(self, i):
        """(weight offset, bias offset) of layer i (0-based; depth = output layer)."""
        return int(self.layout.w_off[i]), int(self.layout.b_off[i])

    def set_params(self, host):
        self.params.copy_(self.torch.as_tensor(np.asarray(host, dtype=np.float32)))
        self.m.zero_()
        self.v.zero_()
        self.iter = 0

    def _ws(self):
        p = self.workspace.data_ptr()
        return C.c_void_p((p + 255) // 256 * 256)

    def forward(self, x, out=None):
        b = int(x.shape[0])
        if b > self.max_batch:
            raise ValueError("batch larger than the workspace")
        out = out if out is not None else self.torch.empty((b, self.desc.d_out),
                                                           dtype=self.torch.float32,
                                                           device=self.device)
        _check(lib.qg_mlp_forward(C.byref(self.desc), self.params.data_ptr(), x.data_ptr(), b,
                                  out.data_ptr(), self._ws(), self._stream()), "qg_mlp_forward")
        return out

    def grad_and_loss(self, x, t):
        b = int(x.shape[0])
        _check(lib.qg_mlp_grad(C.byref(self.desc), self.params.data_ptr(), x.data_ptr(),
                               t.data_ptr(), b, self.grad.data_ptr(), self.loss.data_ptr(),
                               self._ws(), self._stream()), "qg_mlp_grad")
        return self.grad, self.loss[0]

    def train_step(self, x, t, lr):
        b = int(x.shape[0])
        self.iter += 1
        _check(lib.qg_mlp_train_step(C.byref(self.desc), self.params.data_ptr(),
                                     self.m.data_ptr(), self.v.data_ptr(), self.grad.data_ptr(),
                                     x.data_ptr(), t.data_ptr(), b, self.iter, float(lr),
                                     self.loss.data_ptr(), self._ws(), self._stream()),
               "qg_mlp_train_step")
        return self.loss[0]

    def to_bf16(self):
        if self.params16 is None:
            self.params16 = self.torch.empty(self.n_params, dtype=self.torch.int16,
                                             device=self.device)
        _check(lib.qg_mlp_to_bf16(C.byref(self.desc), self.params.data_ptr(),
                                  self.params16.data_ptr(), self._stream()), "qg_mlp_to_bf16")

    def forward_bf16(self, x, out=None):
        b = int(x.shape[0])
        if self.params16 is None:
            self.to_bf16()
        out = out if out is not None else self.torch.empty((b, self.desc.d_out),
                                                           dtype=self.torch.float32,
                                                           device=self.device)
        _check(lib.qg_mlp_forward_bf16(C.byref(self.desc), self.params16.data_ptr(),
                                       x.data_ptr(), b, out.data_ptr(), self._ws(),
                                       self._stream()), "qg_mlp_forward_bf16")
        return out


def batch_bytes(problems):
    """qg_batch_bytes: device bytes of the batch buffer of these problems."""
    n = len(problems)
    out = C.c_size_t(0)
    _check(lib.qg_batch_bytes((_vp * n)(*[C.c_void_p(p.handle.value) for p in problems]), n,
                              C.byref(out)), "qg_batch_bytes")
    return int(out.value)


# batch buffers by device, grown as needed (caller-owned device memory)
_batch_bufs = {}


def solve_batch(problems, xs, ms, vs, opts, cfg=None, stream=None):
    """qg_solve_batch over Problem objects and their device vectors; returns
    the per-scenario reports."""
    import torch
    n = len(problems)
    arr = lambda vals: (_vp * n)(*[C.c_void_p(v) for v in vals])
    reps = (qg_solve_report * n)()
    cfg = cfg or adam_cfg()
    st = stream if stream is not None else torch.cuda.current_stream()
    need = batch_bytes(problems)
    dev = problems[0].device
    buf = _batch_bufs.get(str(dev))
    if buf is None or buf.numel() < need:
        buf = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        _batch_bufs[str(dev)] = buf
    _check(lib.qg_solve_batch(arr([p.handle.value for p in problems]), n,
                              arr([x.data_ptr() for x in xs]), arr([m.data_ptr() for m in ms]),
                              arr([v.data_ptr() for v in vs]),
                              arr([p.workspace.data_ptr() for p in problems]),
                              C.c_void_p(buf.data_ptr()), buf.numel(), C.byref(opts),
                              C.byref(cfg), reps, C.c_void_p(st.cuda_stream)), "qg_solve_batch")
    return list(reps)
