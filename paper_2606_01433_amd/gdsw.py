"""Python binding of the GDSW C ABI (include/gdsw.h): argument marshalling only.

Every numerical step runs in the HIP library libgdsw.so built in this
package directory; PyTorch supplies device memory and the current stream.
There is no CPU fallback: loading fails loudly if the library is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdsw.so")

OK, NOTCONV, EINVAL, ESINGULAR, ENOMEM, EHIP = 0, 1, -1, -2, -3, -4
MAX_RHS = 32          # GDSW_MAX_RHS
_CODE_NAMES = {EINVAL: "EINVAL", ESINGULAR: "ESINGULAR", ENOMEM: "ENOMEM", EHIP: "EHIP", NOTCONV: "NOTCONV"}

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class Problem(ctypes.Structure):
    _fields_ = [("n", c_i64), ("rowptr", c_vp), ("col", c_vp), ("val", c_vp), ("n_nodes", c_i32),
                ("node_dof", c_vp), ("n_elem", c_i32), ("elem_node", c_vp), ("elem_pdof", c_vp),
                ("elem_part", c_vp), ("levels", c_i32), ("n_parts", c_vp), ("part_parent", c_vp)]


class Options(ctypes.Structure):
    _fields_ = [("overlap", c_i32), ("combine", c_i32), ("precision", c_i32), ("restart", c_i32),
                ("max_it", c_i32), ("tol", c_dbl), ("no_coarse", c_i32), ("panel", c_i32), ("profile", c_i32),
                ("graph", c_i32), ("tune", c_i32), ("ls_waves", c_i32), ("lu_variant", c_i32),
                ("pressure_gamma", c_i32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("restarts", c_i32), ("converged", c_i32), ("rel_residual", c_dbl),
                ("ms_apply", c_dbl), ("ms_spmv", c_dbl), ("ms_orth", c_dbl), ("ms_total", c_dbl),
                ("reorthogonalizations", c_i32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", c_i32), ("n", c_i64 * 8), ("parts", c_i32 * 8), ("sum_ni", c_i64 * 8),
                ("max_ni", c_i32 * 8), ("factor_bytes", c_i64 * 8), ("factor_flops", c_dbl * 8),
                ("interior_flops", c_dbl * 8), ("nnz", c_i64 * 8), ("ms_maps", c_dbl), ("ms_extract", c_dbl),
                ("ms_factor", c_dbl), ("ms_basis", c_dbl), ("ms_galerkin", c_dbl), ("ms_coarse", c_dbl),
                ("ms_total", c_dbl), ("local_solve_launches", c_i64), ("ms_local_solve", c_dbl),
                ("local_solve_bytes", c_dbl), ("ls_waves", c_i32 * 8), ("tl_factor", (c_dbl * 2) * 8),
                ("tl_basis", (c_dbl * 2) * 8), ("tl_coarsest", c_dbl * 2), ("ms_lu", c_dbl * 8),
                ("apply_bytes", c_dbl), ("lu_variant", c_i32 * 8), ("local_solve_launches_level", c_i64 * 8),
                ("ms_local_solve_level", c_dbl * 8), ("local_solve_bytes_level", c_dbl * 8),
                ("spmv_bytes", c_dbl)]


class MapsView(ctypes.Structure):
    _fields_ = [("n_dof", c_i32), ("n_parts", c_i32), ("dom_ptr", c_vp), ("dom", c_vp), ("int_ptr", c_vp),
                ("inter", c_vp), ("n_gamma_nodes", c_i32), ("gamma_nodes", c_vp), ("n_entities", c_i32),
                ("ent_ptr", c_vp), ("ent_nodes", c_vp), ("ent_kind", c_vp), ("n_coarse", c_i32),
                ("col_entity", c_vp), ("col_dir", c_vp), ("owner", c_vp)]


# name -> (restype, argtypes); the exact set of functions declared in include/gdsw.h
SIGNATURES = {
    "gdsw_default_options": (None, [ctypes.POINTER(Options)]),
    "gdsw_setup": (c_i32, [ctypes.POINTER(Problem), ctypes.POINTER(Options), c_vp, ctypes.POINTER(c_vp)]),
    "gdsw_apply": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "gdsw_solve": (c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(SolveInfo)]),
    "gdsw_solve_noalloc": (c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(SolveInfo)]),
    "gdsw_apply_multi": (c_i32, [c_vp, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp]),
    "gdsw_solve_multi": (c_i32, [c_vp, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, ctypes.POINTER(SolveInfo)]),
    "gdsw_mg_create": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_dbl,
                                c_vp, ctypes.POINTER(c_vp)]),
    "gdsw_mg_apply": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "gdsw_mg_solve": (c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(SolveInfo)]),
    "gdsw_mg_counts": (c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "gdsw_mg_destroy": (None, [c_vp]),
    "gdsw_spmv": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "gdsw_scatter_local": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "gdsw_export_maps": (c_i32, [c_vp, c_i32, ctypes.POINTER(MapsView)]),
    "gdsw_get_stats": (c_i32, [c_vp, ctypes.POINTER(Stats)]),
    "gdsw_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(Problem), ctypes.POINTER(Options)]),
    "gdsw_plan_create": (c_i32, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(c_vp)]),
    "gdsw_plan_levels": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "gdsw_plan_maps": (c_i32, [c_vp, c_i32, ctypes.POINTER(MapsView)]),
    "gdsw_plan_destroy": (None, [c_vp]),
    "gdsw_destroy": (None, [c_vp]),
    "gdsw_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libgdsw.so (built by paper_2606_01433_amd.build); raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GdswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code < 0:
        raise GdswError(code, load_library().gdsw_last_error().decode())
    return code


def make_options(overlap=1, combine="restricted", precision="fp64", restart=30, max_it=1000, tol=1e-8,
                 no_coarse=False, panel=0, profile=False, graph=False, tune=False, ls_waves=0, lu_variant=0,
                 pressure_gamma="constants"):
    o = Options()
    load_library().gdsw_default_options(ctypes.byref(o))
    o.overlap = overlap
    o.combine = {"restricted": 0, "RAS": 0, "additive": 1, "AS": 1}[combine]
    o.precision = {"fp64": 0, "mixed": 1}[precision]
    o.restart = restart
    o.max_it = max_it
    o.tol = tol
    o.no_coarse = int(bool(no_coarse))
    o.panel = panel
    o.profile = int(bool(profile))
    o.graph = int(bool(graph))
    o.tune = {False: 0, True: 1, "solves": 1, "lu": 2, "all": 3}[tune] if not isinstance(tune, int) or isinstance(tune, bool) else int(tune)
    o.ls_waves = int(ls_waves)
    o.lu_variant = int(lu_variant)
    o.pressure_gamma = {"constants": 0, "all": 1}[pressure_gamma]
    return o


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class _HostArrays:
    """Keeps the host arrays of a Problem alive while the C structure points at them."""

    def __init__(self, p):
        self.node_dof = np.ascontiguousarray(p.node_dof, dtype=np.int32)
        self.elem_node = np.ascontiguousarray(p.elem_node, dtype=np.int32)
        self.elem_pdof = np.ascontiguousarray(p.elem_pdof, dtype=np.int32)
        self.elem_part = np.ascontiguousarray(p.elem_part, dtype=np.int32)
        self.n_parts = np.ascontiguousarray(p.n_parts, dtype=np.int32)
        self.parents = [np.ascontiguousarray(q, dtype=np.int32) for q in p.part_parent]
        self.parent_ptrs = (c_vp * max(1, len(self.parents)))(*[q.ctypes.data for q in self.parents])

    def fill(self, st, p):
        st.n_nodes = int(p.n_nodes)
        st.node_dof = self.node_dof.ctypes.data
        st.n_elem = int(p.n_elem)
        st.elem_node = self.elem_node.ctypes.data
        st.elem_pdof = self.elem_pdof.ctypes.data
        st.elem_part = self.elem_part.ctypes.data
        st.levels = int(p.levels)
        st.n_parts = self.n_parts.ctypes.data
        st.part_parent = ctypes.cast(self.parent_ptrs, c_vp)


def footprint_bytes(problem, **opts):
    """Device bytes a context for this problem would hold (host-only estimate)."""
    lib = load_library()
    st = Problem()
    st.n = int(problem.n)
    h = _HostArrays(problem)
    h.fill(st, problem)
    o = make_options(**opts)
    return int(lib.gdsw_footprint_bytes(ctypes.byref(st), ctypes.byref(o)))


def _view_to_dict(v):
    def arr(ptr, count, ctype):
        if count == 0:
            return np.zeros(0, dtype=np.int64 if ctype is c_i64 else np.int32)
        return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(count,)).copy()
    np_ = v.n_parts
    dom_ptr = arr(v.dom_ptr, np_ + 1, c_i64)
    int_ptr = arr(v.int_ptr, np_ + 1, c_i64)
    ent_ptr = arr(v.ent_ptr, v.n_entities + 1, c_i64)
    return dict(n_dof=v.n_dof, n_parts=np_, dom_ptr=dom_ptr, dom=arr(v.dom, int(dom_ptr[-1]), c_i32),
                int_ptr=int_ptr, inter=arr(v.inter, int(int_ptr[-1]), c_i32),
                gamma_nodes=arr(v.gamma_nodes, v.n_gamma_nodes, c_i32), ent_ptr=ent_ptr,
                ent_nodes=arr(v.ent_nodes, int(ent_ptr[-1]), c_i32),
                ent_kind=arr(v.ent_kind, v.n_entities, c_i32), n_coarse=v.n_coarse,
                col_entity=arr(v.col_entity, v.n_coarse, c_i32), col_dir=arr(v.col_dir, v.n_coarse, c_i32),
                owner=arr(v.owner, v.n_dof, c_i32))


def plan_maps(problem, **opts):
    """Host-only dry run (gdsw_plan_*): index maps of every level, no GPU needed.

    Returns (list of per-level map dicts, has_coarsest)."""
    lib = load_library()
    st = Problem()
    st.n = int(problem.n)
    h = _HostArrays(problem)
    h.fill(st, problem)
    o = make_options(**opts)
    plan = c_vp()
    _check(lib.gdsw_plan_create(ctypes.byref(st), ctypes.byref(o), ctypes.byref(plan)))
    try:
        sl, hc = c_i32(), c_i32()
        _check(lib.gdsw_plan_levels(plan, ctypes.byref(sl), ctypes.byref(hc)))
        out = []
        for lev in range(1, sl.value + 1):
            v = MapsView()
            _check(lib.gdsw_plan_maps(plan, lev, ctypes.byref(v)))
            out.append(_view_to_dict(v))
        return out, bool(hc.value)
    finally:
        lib.gdsw_plan_destroy(plan)


def _check_csr(K, n, dev):
    """The device CSR arrays exactly as gdsw_setup reads them: int64 row pointers (n + 1),
    int32 columns and float64 values of length rowptr[-1], contiguous, on the context's GPU."""
    import torch
    rowptr, col, val = K
    for name, t, dt in (("rowptr", rowptr, torch.int64), ("col", col, torch.int32), ("val", val, torch.float64)):
        if not isinstance(t, torch.Tensor) or t.device != dev or t.dtype != dt or not t.is_contiguous() or t.dim() != 1:
            raise TypeError(f"K.{name} must be a contiguous 1-D {dt} tensor on {dev}")
    if rowptr.numel() != n + 1:
        raise ValueError(f"K.rowptr has {rowptr.numel()} entries, expected n + 1 = {n + 1}")
    nnz = int(rowptr[-1].item())
    if col.numel() != nnz or val.numel() != nnz:
        raise ValueError(f"K.col / K.val have {col.numel()} / {val.numel()} entries, rowptr[-1] = {nnz}")
    return rowptr, col, val


class Context:
    """A built GDSW hierarchy on the current GPU (gdsw_setup ... gdsw_destroy)."""

    def __init__(self, problem, stream=None, K=None, **opts):
        import torch
        lib = load_library()
        self._lib = lib
        self.n = int(problem.n)
        dev = torch.device("cuda", torch.cuda.current_device())
        if K is None:
            K = (torch.as_tensor(np.asarray(problem.rowptr, dtype=np.int64), device=dev),
                 torch.as_tensor(np.asarray(problem.col, dtype=np.int32), device=dev),
                 torch.as_tensor(np.asarray(problem.val, dtype=np.float64), device=dev))
        rowptr, col, val = _check_csr(K, self.n, dev)
        st = Problem()
        st.n = self.n
        st.rowptr, st.col, st.val = rowptr.data_ptr(), col.data_ptr(), val.data_ptr()
        h = _HostArrays(problem)
        h.fill(st, problem)
        self.options = make_options(**opts)
        ctx = c_vp()
        _check(lib.gdsw_setup(ctypes.byref(st), ctypes.byref(self.options), _stream_handle(stream),
                              ctypes.byref(ctx)))
        self._ctx = ctx

    def _alive(self):
        if self._ctx is None:
            raise RuntimeError("context destroyed")
        return self._ctx

    @staticmethod
    def _dev(t, n):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("expected a contiguous CUDA float64 tensor")
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return t.data_ptr()

    def apply(self, r, out=None, stream=None):
        import torch
        z = torch.empty_like(r) if out is None else out
        _check(self._lib.gdsw_apply(self._alive(), self._dev(r, self.n), self._dev(z, self.n),
                                    _stream_handle(stream)))
        return z

    @staticmethod
    def _dev_block(t, n):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.dim() == 2 and t.shape[1] == n):
            raise TypeError(f"expected a contiguous CUDA float64 tensor of shape (k, {n})")
        if not 1 <= t.shape[0] <= MAX_RHS:
            raise ValueError(f"k = {t.shape[0]} right-hand sides, expected 1..{MAX_RHS}")
        return t.data_ptr()

    def apply_multi(self, R, out=None, stream=None):
        """Z[s] = B R[s] for the k rows of R (shape (k, n)): gdsw_apply_multi."""
        import torch
        Z = torch.empty_like(R) if out is None else out
        _check(self._lib.gdsw_apply_multi(self._alive(), int(R.shape[0]), self._dev_block(R, self.n), self.n,
                                          self._dev_block(Z, self.n), self.n, _stream_handle(stream)))
        return Z

    def solve_multi(self, B, out=None, stream=None):
        """k FGMRES solves in lockstep (gdsw_solve_multi); B of shape (k, n). Returns (X, list of infos)."""
        import torch
        X = torch.empty_like(B) if out is None else out
        k = int(B.shape[0])
        infos = (SolveInfo * k)()
        code = _check(self._lib.gdsw_solve_multi(self._alive(), k, self._dev_block(B, self.n), self.n,
                                                 self._dev_block(X, self.n), self.n, _stream_handle(stream), infos))
        out_infos = []
        for q in range(k):
            d = {f: getattr(infos[q], f) for f, _ in SolveInfo._fields_}
            d["code"] = code
            out_infos.append(d)
        return X, out_infos

    def spmv(self, x, out=None, stream=None):
        import torch
        y = torch.empty_like(x) if out is None else out
        _check(self._lib.gdsw_spmv(self._alive(), self._dev(x, self.n), self._dev(y, self.n),
                                   _stream_handle(stream)))
        return y

    def solve(self, b, out=None, stream=None, no_alloc=False):
        """x with ||b - K x|| / ||b|| <= tol (gdsw_solve; no_alloc: gdsw_solve_noalloc, whose
        workspace is the library's static device array)."""
        import torch
        x = torch.empty_like(b) if out is None else out
        info = SolveInfo()
        fn = self._lib.gdsw_solve_noalloc if no_alloc else self._lib.gdsw_solve
        code = _check(fn(self._alive(), self._dev(b, self.n), self._dev(x, self.n), _stream_handle(stream),
                         ctypes.byref(info)))
        d = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        d["code"] = code
        return x, d

    def scatter_local(self, level, w, out=None, stream=None):
        import torch
        maps = self.export_maps(level)
        z = torch.empty(maps["n_dof"], dtype=torch.float64, device=w.device) if out is None else out
        _check(self._lib.gdsw_scatter_local(self._alive(), int(level), self._dev(w, int(maps["dom_ptr"][-1])),
                                            self._dev(z, maps["n_dof"]), _stream_handle(stream)))
        return z

    def export_maps(self, level):
        v = MapsView()
        _check(self._lib.gdsw_export_maps(self._alive(), int(level), ctypes.byref(v)))
        return _view_to_dict(v)

    def stats(self):
        s = Stats()
        _check(self._lib.gdsw_get_stats(self._alive(), ctypes.byref(s)))
        out = {}
        for k, t in Stats._fields_:
            v = getattr(s, k)
            if hasattr(t, "_length_"):
                v = [list(x) if hasattr(x, "_length_") else x for x in v]
            out[k] = v
        return out

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            self._lib.gdsw_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class MultiGrid:
    """Two-grid geometric multigrid with the GDSW solver as coarse solver (gdsw_mg_*).

    fine: Context on the fine problem (its apply is the smoother, its operator K_f);
    coarse: Context on the coarse problem (its tol is the coarse reduction);
    P: scipy sparse prolongation (fine free dofs x coarse free dofs)."""

    def __init__(self, fine, coarse, P, nu_pre=2, nu_post=2, omega=1.0, stream=None):
        import torch
        lib = load_library()
        self._lib = lib
        self.fine, self.coarse = fine, coarse
        self.n = fine.n
        dev = torch.device("cuda", torch.cuda.current_device())
        P = P.tocsr()
        PT = P.T.tocsr()
        P.sort_indices()
        PT.sort_indices()
        self._arrays = []
        ptrs = []
        for M in (P, PT):
            t = (torch.as_tensor(M.indptr.astype(np.int64), device=dev),
                 torch.as_tensor(M.indices.astype(np.int32), device=dev),
                 torch.as_tensor(M.data.astype(np.float64), device=dev))
            self._arrays.append(t)
            ptrs.extend(x.data_ptr() for x in t)
        out = c_vp()
        _check(lib.gdsw_mg_create(fine._alive(), coarse._alive(), fine.n, coarse.n, *ptrs, int(nu_pre), int(nu_post),
                                  float(omega), _stream_handle(stream), ctypes.byref(out)))
        self._mg = out

    def apply(self, r, out=None, stream=None):
        import torch
        z = torch.empty_like(r) if out is None else out
        _check(self._lib.gdsw_mg_apply(self._mg, Context._dev(r, self.n), Context._dev(z, self.n),
                                       _stream_handle(stream)))
        return z

    def solve(self, b, out=None, stream=None):
        import torch
        x = torch.empty_like(b) if out is None else out
        info = SolveInfo()
        code = _check(self._lib.gdsw_mg_solve(self._mg, Context._dev(b, self.n), Context._dev(x, self.n),
                                              _stream_handle(stream), ctypes.byref(info)))
        d = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        d["code"] = code
        return x, d

    def counts(self):
        c, k = c_i64(), c_i64()
        _check(self._lib.gdsw_mg_counts(self._mg, ctypes.byref(c), ctypes.byref(k)))
        return {"cycles": c.value, "coarse_iterations": k.value}

    def close(self):
        if getattr(self, "_mg", None) is not None:
            self._lib.gdsw_mg_destroy(self._mg)
            self._mg = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
