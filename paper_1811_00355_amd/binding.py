"""ctypes binding of libdd (include/dd.h).  Argument marshalling only: every
operation runs in the HIP library.  Device buffers are torch tensors on the
GPU (their data pointers are passed through); streams are torch streams.

The library must have been built (paper_1811_00355_amd/build.py); importing
this module fails loudly when it is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdd.so")

DD_F64, DD_F32, DD_F16, DD_BF16 = 0, 1, 2, 3
DTYPES = {"f64": DD_F64, "f32": DD_F32, "f16": DD_F16, "bf16": DD_BF16}
STATUS = ["DD_OK", "DD_EINVAL", "DD_ESHAPE", "DD_ENOMEM", "DD_EBUDGET", "DD_ENOCONV",
          "DD_ENAN", "DD_EDEVICE", "DD_ESTATE"]


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else str(status)


class dd_problem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("block", ctypes.c_int32 * 4), ("bc_t", ctypes.c_int32),
                ("m0", ctypes.c_double), ("c_sw", ctypes.c_double)]


class dd_mg_params(ctypes.Structure):
    _fields_ = [("agg_block", ctypes.c_int32 * 4), ("sap_block", ctypes.c_int32 * 4),
                ("n_vec", ctypes.c_int32), ("setup_iters", ctypes.c_int32),
                ("init_sap_apps", ctypes.c_int32), ("sap_sweeps", ctypes.c_int32),
                ("sap_mr_iters", ctypes.c_int32), ("coarse_restart", ctypes.c_int32),
                ("coarse_max_iters", ctypes.c_int32), ("coarse_fixed_iters", ctypes.c_int32),
                ("fgmres_restart", ctypes.c_int32), ("max_outer_iters", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double), ("inner_dtype", ctypes.c_int32),
                ("store_dtype", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("coarse_cgs_passes", ctypes.c_int32), ("outer_cgs_passes", ctypes.c_int32)]


class dd_tuning(ctypes.Structure):
    _fields_ = [("sap_wpe", ctypes.c_int32), ("dirac_threads", ctypes.c_int32), ("coarse_spw", ctypes.c_int32),
                ("coarse_half", ctypes.c_int32), ("coarse_basis_half", ctypes.c_int32),
                ("coarse_mfma_half", ctypes.c_int32), ("sap_dom_rhs", ctypes.c_int32),
                ("sap_persist", ctypes.c_int32)]


class dd_bicgstab_params(ctypes.Structure):
    _fields_ = [("sap_sweeps", ctypes.c_int32), ("sap_mr_iters", ctypes.c_int32),
                ("inner_max_iters", ctypes.c_int32), ("max_outer_iters", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("store_dtype", ctypes.c_int32), ("use_x0", ctypes.c_int32)]


class dd_solve_info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("coarse_iters_total", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("true_relres", ctypes.c_double), ("t_setup_s", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("bytes_model", ctypes.c_int64),
                ("flops_model", ctypes.c_int64)]


class dd_level3_params(ctypes.Structure):
    _fields_ = [("n_vec2", ctypes.c_int32), ("setup_iters", ctypes.c_int32), ("mr_steps", ctypes.c_int32),
                ("kcycle_max_iters", ctypes.c_int32), ("kcycle_fixed", ctypes.c_int32),
                ("l3_restart", ctypes.c_int32), ("l3_max_iters", ctypes.c_int32), ("l3_fixed_iters", ctypes.c_int32),
                ("kcycle_tol", ctypes.c_double), ("l3_tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class dd_footprint(ctypes.Structure):
    _fields_ = [("gauge_bytes", ctypes.c_size_t), ("setup_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_S = ctypes.c_size_t

# name -> (restype, argtypes); every symbol declared in include/dd.h
SIGNATURES = {
    "dd_ctx_create": (_I, [_I, _S, ctypes.POINTER(_P)]),
    "dd_ctx_destroy": (None, [_P]),
    "dd_status_str": (ctypes.c_char_p, [_I]),
    "dd_last_error": (ctypes.c_char_p, [_P]),
    "dd_ctx_bytes_in_use": (_S, [_P]),
    "dd_mg_params_default": (None, [ctypes.POINTER(dd_mg_params)]),
    "dd_gauge_create": (_I, [_P, ctypes.POINTER(dd_problem), _P, ctypes.POINTER(_P)]),
    "dd_gauge_destroy": (_I, [_P]),
    "dd_gauge_set_mass": (_I, [_P, ctypes.c_double]),
    "dd_fine_vec_bytes": (_S, [_P, _I, _I]),
    "dd_coarse_vec_bytes": (_S, [_P, _I, _I]),
    "dd_pack_fine": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_unpack_fine": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_pack_coarse": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_unpack_coarse": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_dirac_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_sap_smooth": (_I, [_P, ctypes.POINTER(dd_mg_params), _I, _I, _P, _P, _P]),
    "dd_setup": (_I, [_P, ctypes.POINTER(dd_mg_params), ctypes.POINTER(_P)]),
    "dd_setup_from_vectors": (_I, [_P, ctypes.POINTER(dd_mg_params), _P, ctypes.POINTER(_P)]),
    "dd_mg_destroy": (_I, [_P]),
    "dd_setup_update_mass": (_I, [_P, ctypes.c_double]),
    "dd_mg_set_graphs": (_I, [_P, _I]),
    "dd_bicgstab_params_default": (None, [ctypes.POINTER(dd_bicgstab_params)]),
    "dd_solve_bicgstab": (_I, [_P, ctypes.POINTER(dd_bicgstab_params), _I, _P, _P, ctypes.c_double,
                               ctypes.POINTER(dd_solve_info), _P]),
    "dd_mg_release_workspace": (_I, [_P]),
    "dd_footprint_bytes": (_I, [ctypes.POINTER(dd_problem), ctypes.POINTER(dd_mg_params), _I,
                                ctypes.POINTER(dd_footprint)]),
    "dd_autotune": (_I, [_P, _I, ctypes.c_char_p, ctypes.c_char_p, _S]),
    "dd_gauge_set_tuning": (_I, [_P, ctypes.POINTER(dd_tuning)]),
    "dd_gauge_get_tuning": (_I, [_P, ctypes.POINTER(dd_tuning)]),
    "dd_restrict": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_prolong": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_coarse_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "dd_coarse_solve": (_I, [_P, _I, _I, _P, _P, ctypes.POINTER(_I), _P]),
    "dd_coarse_solve_noalloc": (_I, [_P, _I, _I, _P, _P, ctypes.POINTER(_I), _P]),
    "dd_precond_apply": (_I, [_P, _I, _P, _P, _P]),
    "dd_solve": (_I, [_P, _I, _P, _P, ctypes.c_double, ctypes.POINTER(dd_solve_info), _P]),
    "dd_solve_begin": (_I, [_P, _I, ctypes.c_double, _P, ctypes.POINTER(_P)]),
    "dd_solve_add": (_I, [_P, _I, _P]),
    "dd_solve_step": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "dd_solve_take": (_I, [_P, _I, _P, ctypes.POINTER(dd_solve_info)]),
    "dd_solve_end": (_I, [_P]),
    "dd_export_maps": (_I, [_P, _P, _P, _P, _P]),
    "dd_export_clover": (_I, [_P, _P, _P]),
    "dd_export_operands": (_I, [_P, _I, _P, _P]),
    "dd_export_coarse": (_I, [_P, _P]),
    "dd_level3_params_default": (None, [ctypes.POINTER(dd_level3_params)]),
    "dd_mg_add_level": (_I, [_P, ctypes.POINTER(dd_level3_params), _P]),
    "dd_mg_remove_level": (_I, [_P]),
    "dd_level3_shape": (_I, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "dd_level3_last": (_I, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "dd_export_level3": (_I, [_P, _P, _P, _P]),
    "dd_export_vectors": (_I, [_P, _P]),
    "dd_kernel_timer_enable": (_I, [ctypes.c_char_p]),
    "dd_kernel_timer_read": (_I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "dd_kernel_timer_names": (_I, [ctypes.c_char_p, ctypes.c_size_t]),
}


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                paths.add(parts[-1])
    return paths


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libdd is not built ({path} missing): run paper_1811_00355_amd/build.py")
    # torch brings its own HIP runtime; load it first so that libdd binds to the
    # same runtime (one HIP runtime per process; the soname matches).
    import torch  # noqa: F401
    import torch.cuda  # noqa: F401
    lib = ctypes.CDLL(path)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes mapped into the process: {sorted(rts)}")
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, device=0, hbm_budget_bytes=200 << 30):
        self.h = _P()
        self.lib = lib()
        st = self.lib.dd_ctx_create(device, hbm_budget_bytes, ctypes.byref(self.h))
        if st:
            raise DDError(st, "dd_ctx_create failed")

    def check(self, st):
        if st:
            raise DDError(st, self.lib.dd_last_error(self.h).decode())

    def bytes_in_use(self):
        return self.lib.dd_ctx_bytes_in_use(self.h)

    def close(self):
        if self.h:
            self.lib.dd_ctx_destroy(self.h)
            self.h = _P()


def bicgstab_params(**kw):
    p = dd_bicgstab_params()
    lib().dd_bicgstab_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def footprint(L, block, params, nrhs, bc_t=-1):
    """Device bytes the library allocates for this shape (dd_footprint_bytes):
    dict with gauge, setup, scratch and workspace figures.  Host arithmetic only."""
    prob = dd_problem((ctypes.c_int32 * 4)(*L), (ctypes.c_int32 * 4)(*block), bc_t, 0.0, 1.0)
    out = dd_footprint()
    st = lib().dd_footprint_bytes(ctypes.byref(prob), ctypes.byref(params), nrhs, ctypes.byref(out))
    if st:
        raise DDError(st, f"dd_footprint_bytes(L={tuple(L)}, block={tuple(block)}, nrhs={nrhs})")
    return dict(gauge=out.gauge_bytes, setup=out.setup_bytes, scratch=out.scratch_bytes,
                workspace=out.workspace_bytes)


def default_params(**kw):
    p = dd_mg_params()
    lib().dd_mg_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("agg_block", "sap_block", "block"):
            for m in range(4):
                if k in ("agg_block", "block"):
                    p.agg_block[m] = v[m]
                if k in ("sap_block", "block"):
                    p.sap_block[m] = v[m]
        else:
            setattr(p, k, v)
    return p


def level3_params(**kw):
    p = dd_level3_params()
    lib().dd_level3_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Gauge:
    """A gauge field on the device: links, clover, clover inverse."""

    def __init__(self, ctx, L, block, links, m0, c_sw, bc_t=-1):
        self.ctx = ctx
        self.L, self.block = tuple(L), tuple(block)
        self.V = int(np.prod(L))
        self.Vc = int(np.prod([L[m] // block[m] for m in range(4)]))
        pr = dd_problem()
        for m in range(4):
            pr.L[m] = L[m]
            pr.block[m] = block[m]
        pr.bc_t, pr.m0, pr.c_sw = bc_t, m0, c_sw
        links = np.ascontiguousarray(links, dtype=np.complex128)
        assert links.shape == (self.V, 4, 3, 3)
        self.h = _P()
        ctx.check(ctx.lib.dd_gauge_create(ctx.h, ctypes.byref(pr), links.ctypes.data_as(_P), ctypes.byref(self.h)))

    def destroy(self):
        if self.h:
            self.ctx.check(self.ctx.lib.dd_gauge_destroy(self.h))
            self.h = _P()

    def dd_gauge_set_tuning(self, sap_wpe, dirac_threads, coarse_spw, coarse_half=0, coarse_basis_half=0,
                            coarse_mfma_half=0, sap_dom_rhs=2, sap_persist=0):
        t = dd_tuning(sap_wpe, dirac_threads, coarse_spw, coarse_half, coarse_basis_half, coarse_mfma_half,
                      sap_dom_rhs, sap_persist)
        self.ctx.check(self.ctx.lib.dd_gauge_set_tuning(self.h, ctypes.byref(t)))

    def dd_gauge_get_tuning(self):
        t = dd_tuning()
        self.ctx.check(self.ctx.lib.dd_gauge_get_tuning(self.h, ctypes.byref(t)))
        return dict(sap_wpe=t.sap_wpe, dirac_threads=t.dirac_threads, coarse_spw=t.coarse_spw,
                    coarse_half=t.coarse_half, coarse_basis_half=t.coarse_basis_half,
                    coarse_mfma_half=t.coarse_mfma_half, sap_dom_rhs=t.sap_dom_rhs, sap_persist=t.sap_persist)

    def dd_solve_bicgstab(self, params, nrhs, b_canon, x_canon, tol, stream=None, raise_on_noconv=True):
        """The paper's comparison solver (SAP-preconditioned FP32 BiCGstab in an FP64 defect correction)."""
        info = (dd_solve_info * nrhs)()
        st = self.ctx.lib.dd_solve_bicgstab(self.h, ctypes.byref(params), nrhs, _ptr(b_canon), _ptr(x_canon), tol, info,
                                            _stream(stream))
        if st and not (st == 5 and not raise_on_noconv):
            self.ctx.check(st)
        return [dict(outer_iters=i.outer_iters, inner_iters=i.coarse_iters_total, converged=bool(i.converged),
                     true_relres=i.true_relres, t_solve_s=i.t_solve_s) for i in info], st

    def dd_gauge_set_mass(self, m0):
        self.ctx.check(self.ctx.lib.dd_gauge_set_mass(self.h, m0))

    # vectors ---------------------------------------------------------------------------
    def fine_vec_bytes(self, dtype, nrhs):
        return self.ctx.lib.dd_fine_vec_bytes(self.h, dtype, nrhs)

    def new_packed(self, dtype, nrhs, device="cuda"):
        import torch
        nb = self.fine_vec_bytes(dtype, nrhs)
        return torch.zeros(nb, dtype=torch.uint8, device=device)

    def pack(self, dtype, nrhs, canon, packed, stream=None):
        self.ctx.check(self.ctx.lib.dd_pack_fine(self.h, dtype, nrhs, _ptr(canon), _ptr(packed), _stream(stream)))

    def unpack(self, dtype, nrhs, packed, canon, stream=None):
        self.ctx.check(self.ctx.lib.dd_unpack_fine(self.h, dtype, nrhs, _ptr(packed), _ptr(canon), _stream(stream)))

    # operations ------------------------------------------------------------------------
    def dd_dirac_apply(self, dtype, nrhs, inp, out, stream=None):
        self.ctx.check(self.ctx.lib.dd_dirac_apply(self.h, dtype, nrhs, _ptr(inp), _ptr(out), _stream(stream)))

    def dd_sap_smooth(self, params, dtype, nrhs, b, x, stream=None):
        self.ctx.check(self.ctx.lib.dd_sap_smooth(self.h, ctypes.byref(params), dtype, nrhs, _ptr(b), _ptr(x),
                                                  _stream(stream)))

    def export_maps(self):
        agg = np.zeros(self.V, np.int32)
        loc = np.zeros(self.V, np.int32)
        pidx = np.zeros(self.V, np.int32)
        col = np.zeros(self.Vc, np.int8)
        self.ctx.check(self.ctx.lib.dd_export_maps(self.h, agg.ctypes.data_as(_P), loc.ctypes.data_as(_P),
                                                   pidx.ctypes.data_as(_P), col.ctypes.data_as(_P)))
        return agg, loc, pidx, col

    def export_operands(self, dtype):
        """Raw stored links [36][V] and clover [36][V] pairs of `dtype`, packed site order."""
        pair = {DD_F64: np.complex128, DD_F32: np.complex64, DD_F16: np.uint32, DD_BF16: np.uint32}[dtype]
        links = np.zeros((36, self.V), dtype=pair)
        clov = np.zeros((36, self.V), dtype=pair)
        self.ctx.check(self.ctx.lib.dd_export_operands(self.h, dtype, links.ctypes.data_as(_P),
                                                       clov.ctypes.data_as(_P)))
        return links, clov

    def export_clover(self):
        a = np.zeros((self.V, 2, 36))
        ai = np.zeros((self.V, 2, 36))
        self.ctx.check(self.ctx.lib.dd_export_clover(self.h, a.ctypes.data_as(_P), ai.ctypes.data_as(_P)))
        return a, ai


class MG:
    """A two-level multigrid setup on a gauge field."""

    def __init__(self, gauge, params, tv_host=None):
        self.g = gauge
        self.ctx = gauge.ctx
        self.p = params
        self.n = params.n_vec
        self.h = _P()
        if tv_host is None:
            self.ctx.check(self.ctx.lib.dd_setup(gauge.h, ctypes.byref(params), ctypes.byref(self.h)))
        else:
            tv = np.ascontiguousarray(tv_host, dtype=np.complex128)
            assert tv.shape == (self.n, gauge.V, 4, 3)
            self.ctx.check(self.ctx.lib.dd_setup_from_vectors(gauge.h, ctypes.byref(params), tv.ctypes.data_as(_P),
                                                              ctypes.byref(self.h)))

    def destroy(self):
        if self.h:
            self.ctx.check(self.ctx.lib.dd_mg_destroy(self.h))
            self.h = _P()

    def dd_autotune(self, nrhs, cache_path=None):
        """Time the launch-shape candidates, keep the fastest; returns the report text."""
        buf = ctypes.create_string_buffer(4096)
        path = None if cache_path is None else os.fsencode(cache_path)
        self.ctx.check(self.ctx.lib.dd_autotune(self.h, nrhs, path, buf, len(buf)))
        return buf.value.decode()

    def dd_mg_release_workspace(self):
        self.ctx.check(self.ctx.lib.dd_mg_release_workspace(self.h))

    def dd_mg_set_graphs(self, mode):
        """0: launches; 1: coarse GMRES chunks from graphs; 2: all of M from one graph (True means 1)."""
        self.ctx.check(self.ctx.lib.dd_mg_set_graphs(self.h, int(mode)))

    def dd_setup_update_mass(self, m0):
        self.ctx.check(self.ctx.lib.dd_setup_update_mass(self.h, m0))

    def coarse_vec_bytes(self, dtype, nrhs):
        return self.ctx.lib.dd_coarse_vec_bytes(self.h, dtype, nrhs)

    def new_coarse(self, dtype, nrhs, device="cuda"):
        import torch
        return torch.zeros(self.coarse_vec_bytes(dtype, nrhs), dtype=torch.uint8, device=device)

    def pack_coarse(self, dtype, nrhs, canon, packed, stream=None):
        self.ctx.check(self.ctx.lib.dd_pack_coarse(self.h, dtype, nrhs, _ptr(canon), _ptr(packed), _stream(stream)))

    def unpack_coarse(self, dtype, nrhs, packed, canon, stream=None):
        self.ctx.check(self.ctx.lib.dd_unpack_coarse(self.h, dtype, nrhs, _ptr(packed), _ptr(canon),
                                                     _stream(stream)))

    def dd_restrict(self, dtype, nrhs, fine, coarse, stream=None):
        self.ctx.check(self.ctx.lib.dd_restrict(self.h, dtype, nrhs, _ptr(fine), _ptr(coarse), _stream(stream)))

    def dd_prolong(self, dtype, nrhs, coarse, fine, stream=None):
        self.ctx.check(self.ctx.lib.dd_prolong(self.h, dtype, nrhs, _ptr(coarse), _ptr(fine), _stream(stream)))

    def dd_coarse_apply(self, dtype, nrhs, inp, out, stream=None):
        self.ctx.check(self.ctx.lib.dd_coarse_apply(self.h, dtype, nrhs, _ptr(inp), _ptr(out), _stream(stream)))

    def dd_coarse_solve(self, dtype, nrhs, inp, out, stream=None):
        it = _I(0)
        self.ctx.check(self.ctx.lib.dd_coarse_solve(self.h, dtype, nrhs, _ptr(inp), _ptr(out), ctypes.byref(it),
                                                    _stream(stream)))
        return it.value

    def dd_coarse_solve_noalloc(self, dtype, nrhs, inp, out, stream=None):
        """dd_coarse_solve on the library's static scratch (no device allocation)."""
        it = _I(0)
        self.ctx.check(self.ctx.lib.dd_coarse_solve_noalloc(self.h, dtype, nrhs, _ptr(inp), _ptr(out),
                                                            ctypes.byref(it), _stream(stream)))
        return it.value

    def dd_precond_apply(self, nrhs, inp, out, stream=None):
        self.ctx.check(self.ctx.lib.dd_precond_apply(self.h, nrhs, _ptr(inp), _ptr(out), _stream(stream)))

    def dd_solve(self, nrhs, b_canon, x_canon, tol, stream=None, raise_on_noconv=True):
        info = (dd_solve_info * nrhs)()
        st = self.ctx.lib.dd_solve(self.h, nrhs, _ptr(b_canon), _ptr(x_canon), tol, info, _stream(stream))
        if st and not (st == 5 and not raise_on_noconv):
            self.ctx.check(st)
        return [_info_dict(i) for i in info], st

    def dd_solve_begin(self, capacity, tol, stream=None):
        """A stepwise solve with `capacity` slots on this multigrid's workspace."""
        return SolveState(self, capacity, tol, stream)

    def export_coarse(self):
        nc = 2 * self.n
        dc = np.zeros((self.g.Vc, 9, nc, nc), dtype=np.complex128)
        self.ctx.check(self.ctx.lib.dd_export_coarse(self.h, dc.ctypes.data_as(_P)))
        return dc

    def export_vectors(self):
        tv = np.zeros((self.n, self.g.V, 4, 3), dtype=np.complex128)
        self.ctx.check(self.ctx.lib.dd_export_vectors(self.h, tv.ctypes.data_as(_P)))
        return tv

    def add_level(self, params, tv2_host=None):
        """Attach the third level; tv2_host: None or [n_vec2][Vc][2n] complex128 (coarse sites lexicographic)."""
        if tv2_host is None:
            self.ctx.check(self.ctx.lib.dd_mg_add_level(self.h, ctypes.byref(params), None))
        else:
            tv = np.ascontiguousarray(tv2_host, dtype=np.complex128)
            assert tv.shape == (params.n_vec2, self.g.Vc, 2 * self.n)
            self.ctx.check(self.ctx.lib.dd_mg_add_level(self.h, ctypes.byref(params), tv.ctypes.data_as(_P)))

    def remove_level(self):
        self.ctx.check(self.ctx.lib.dd_mg_remove_level(self.h))

    def level3_shape(self):
        """(Vc3, nc3): level-3 sites and components per site; (0, 0) without a third level."""
        a, b = ctypes.c_int32(0), ctypes.c_int32(0)
        self.ctx.check(self.ctx.lib.dd_level3_shape(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def level3_last(self):
        """(level-2 FGMRES steps, level-3 GMRES steps) of the last coarse solve."""
        a, b = ctypes.c_int32(0), ctypes.c_int32(0)
        self.ctx.check(self.ctx.lib.dd_level3_last(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def export_level3(self):
        """(tv2 [n2][Vc][2n], P2 [Vc3][2][n2][16 n], D3 [Vc3][9][nc3][nc3]), complex128, lexicographic sites."""
        vc3, nc3 = self.level3_shape()
        n2 = nc3 // 2
        tv2 = np.zeros((n2, self.g.Vc, 2 * self.n), dtype=np.complex128)
        p2 = np.zeros((vc3, 2, n2, 16 * self.n), dtype=np.complex128)
        d3 = np.zeros((vc3, 9, nc3, nc3), dtype=np.complex128)
        self.ctx.check(self.ctx.lib.dd_export_level3(self.h, tv2.ctypes.data_as(_P), p2.ctypes.data_as(_P),
                                                     d3.ctypes.data_as(_P)))
        return tv2, p2, d3


def _info_dict(i):
    return dict(outer_iters=i.outer_iters, restarts=i.restarts, coarse_iters_total=i.coarse_iters_total,
                converged=bool(i.converged), true_relres=i.true_relres, t_setup_s=i.t_setup_s,
                t_solve_s=i.t_solve_s, bytes_model=i.bytes_model, flops_model=i.flops_model)


SLOT_FREE, SLOT_RUNNING, SLOT_DONE = 0, 1, 2


class SolveState:
    """dd_solve_begin / add / step / take / end: FGMRES driven one restart
    cycle at a time, right-hand sides admitted into free slots between steps."""

    def __init__(self, mg, capacity, tol, stream=None):
        self.mg, self.ctx, self.capacity = mg, mg.ctx, capacity
        self.stream = stream
        self.h = _P()
        self.ctx.check(self.ctx.lib.dd_solve_begin(mg.h, capacity, tol, _stream(stream), ctypes.byref(self.h)))
        self.states = (ctypes.c_int32 * capacity)()

    def add(self, slot, b_canon):
        """Start `slot` from x = 0 on b (canonical complex128 device vector of one right-hand side)."""
        self.ctx.check(self.ctx.lib.dd_solve_add(self.h, slot, _ptr(b_canon)))

    def step(self):
        """One restart cycle, then the residual check; returns the slot states (0 free, 1 running, 2 done)."""
        self.ctx.check(self.ctx.lib.dd_solve_step(self.h, self.states))
        return list(self.states)

    def take(self, slot, x_canon):
        info = dd_solve_info()
        self.ctx.check(self.ctx.lib.dd_solve_take(self.h, slot, _ptr(x_canon), ctypes.byref(info)))
        return _info_dict(info)

    def end(self):
        if self.h:
            self.ctx.check(self.ctx.lib.dd_solve_end(self.h))
            self.h = _P()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.end()


def kernel_timer_enable(name="*"):
    lib().dd_kernel_timer_enable(None if name is None else name.encode())


def kernel_timer_read(name):
    ms, n, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    st = lib().dd_kernel_timer_read(name.encode(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by), ctypes.byref(fl))
    if st:
        raise DDError(st, "dd_kernel_timer_read failed")
    return dict(ms=ms.value, launches=n.value, bytes=by.value, flops=fl.value)


def kernel_timer_names():
    buf = ctypes.create_string_buffer(4096)
    lib().dd_kernel_timer_names(buf, 4096)
    v = buf.value.decode()
    return v.split(";") if v else []
