"""MI355X (gfx950) multilevel Monte-Carlo estimation of tr(A^{-1}).

Thin Python binding of the C ABI in include/mlmc.h.  Every step of the method
runs in the HIP library libmlmc.so; this module only marshals arguments,
passes torch's device memory and stream, and converts results.  If the library
has not been built, importing the binding raises: there is no CPU fallback.
"""
import atexit
import ctypes
import sys
import weakref

import numpy as np

from . import _capi
from ._capi import (ALLOC_EQUAL, ALLOC_GILES, ALLOC_WEIGHTS, CSR, FP32_IR64,  # noqa: F401
                    FP64, GAUGE2D, POISSON2D, VARCOEF3D, WILSON2D)

KINDS = {"poisson2d": POISSON2D, "wilson2d": WILSON2D, "varcoef3d": VARCOEF3D, "csr": CSR,
         "gauge2d": GAUGE2D}
PRECISIONS = {"fp64": FP64, "fp32_ir64": FP32_IR64}
ALLOCS = {"equal": ALLOC_EQUAL, "weights": ALLOC_WEIGHTS, "giles": ALLOC_GILES}


class MLMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_status(code), code, msg))
        self.code = code


def lib():
    return _capi.load()


def _status(code):
    return lib().mlmc_status_string(code).decode()


def _check(rc, ctx=None):
    if rc != 0:
        msg = lib().mlmc_last_error(ctx)
        raise MLMCError(rc, msg.decode() if msg else "")


def default_options():
    o = _capi.Options()
    _check(lib().mlmc_default_options(ctypes.byref(o)))
    return o


def _result_dict(r):
    L = max(r.levels, 1)
    nl = L - 1 if L > 1 else 1
    return dict(
        trace=complex(r.trace[0], r.trace[1]), rmsd=r.rmsd, tau=r.tau,
        coarse=complex(r.coarse_trace[0], r.coarse_trace[1]), levels=r.levels,
        n_samples=[int(r.n_samples[i]) for i in range(nl)],
        level_mean=[complex(r.level_mean[i][0], r.level_mean[i][1]) for i in range(nl)],
        level_var=[r.level_var[i] for i in range(nl)],
        level_cost=[r.level_cost[i] for i in range(nl)],
        level_seconds=[r.level_seconds[i] for i in range(nl)],
        solves=int(r.solves), iterations=int(r.iterations), seconds=r.seconds)


# ---------------------------------------------------------------------------
# torch's caching allocator as the library's device allocator
# ---------------------------------------------------------------------------
_alloc_refs = []   # the ctypes thunks live for the whole process


def use_torch_allocator(enable=True):
    """Route the library's device allocations through torch's caching allocator.

    The callbacks are created once per process and never replaced: contexts
    keep the function pointers they were created with and call them when they
    are destroyed.
    """
    if not enable:
        _check(lib().mlmc_set_allocator(_capi.ALLOC_FN(0), _capi.FREE_FN(0), None))
        return
    if not _alloc_refs:
        import torch

        def _alloc(nbytes, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:  # reported to the library as a failed allocation
                return None

        def _free(ptr, _user):
            torch.cuda.caching_allocator_delete(ptr)

        _alloc_refs[:] = [_capi.ALLOC_FN(_alloc), _capi.FREE_FN(_free)]
    _check(lib().mlmc_set_allocator(_alloc_refs[0], _alloc_refs[1], None))


_live = weakref.WeakSet()  # open estimators, closed at interpreter exit
_exit_hook = []


def _close_live():
    # runs while the interpreter, torch and the allocator thunks are intact, so
    # a context freeing its device memory through the thunks is still safe
    for est in list(_live):
        est.close()


class TraceEstimator:
    """One operator, its hierarchy and the solvers on the current torch device.

    kind: "poisson2d" | "wilson2d" | "gauge2d" | "varcoef3d" | "csr"; field:
    numpy array of link phases (wilson2d, gauge2d) or face coefficients
    (varcoef3d); matrix: the csr
    kind's matrix (anything with indptr, indices and data after .tocsr(), e.g.
    a scipy.sparse matrix; n_side is ignored); agg: optional aggregate maps of
    the csr kind, one integer array per level below the coarsest (None: greedy
    aggregation in the library); prolongations: the csr kind's P_l (scipy sparse,
    n_l x n_{l+1}; R_l = P_l^T, general decomposition with finest-level
    probes); spin_split: the spin-structure-preserving
    aggregation of the wilson2d kind.  Options follow mlmc_options
    (include/mlmc.h); unknown keyword names raise.
    """

    def __init__(self, kind, n_side, levels_solver, levels_mlmc=None, *, diag=4.0, off=1.0,
                 mass=0.0, shift=0.0, field=None, matrix=None, agg=None, prolongations=None,
                 block=4, n_vec=8, setup_sweeps=20, setup_seed=1, spin_split=False, stream=None,
                 torch_allocator=True, **options):
        import torch
        self._lib = lib()
        self._ctx = ctypes.c_void_p()
        if torch_allocator:
            use_torch_allocator(True)
        op = _capi.Operator()
        op.kind = KINDS[kind]
        op.n_side = int(n_side)
        op.diag, op.off, op.mass, op.shift = float(diag), float(off), float(mass), float(shift)
        self._field = None
        if field is not None:
            self._field = np.ascontiguousarray(field, dtype=np.float64)
            N = int(n_side)
            want = {"wilson2d": 2 * N * N, "gauge2d": 2 * N * N,
                    "varcoef3d": 3 * N * N * (N + 1)}.get(kind)
            if want is not None and self._field.size != want:
                raise ValueError("%s field must hold %d values, got %d"
                                 % (kind, want, self._field.size))
            op.field = self._field.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if matrix is not None:
            m = matrix.tocsr() if hasattr(matrix, "tocsr") else matrix
            self._csr = (np.ascontiguousarray(m.indptr, dtype=np.int64),
                         np.ascontiguousarray(m.indices, dtype=np.int32),
                         np.ascontiguousarray(m.data, dtype=np.float64))
            op.n = len(self._csr[0]) - 1
            op.row_ptr = self._csr[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            op.col_idx = self._csr[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            op.vals = self._csr[2].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = _capi.Hierarchy()
        h.levels_solver = int(levels_solver)
        h.levels_mlmc = int(levels_mlmc if levels_mlmc is not None else levels_solver)
        h.block, h.n_vec, h.setup_sweeps = int(block), int(n_vec), int(setup_sweeps)
        h.setup_seed = int(setup_seed)
        h.spin_split = 1 if spin_split else 0
        if agg is not None:
            self._agg = [np.ascontiguousarray(a, dtype=np.int32) for a in agg]
            if len(self._agg) != h.levels_solver - 1:
                raise ValueError("agg needs levels_solver - 1 maps, got %d" % len(self._agg))
            self._agg_ptrs = (ctypes.POINTER(ctypes.c_int32) * len(self._agg))(
                *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in self._agg])
            h.agg = ctypes.cast(self._agg_ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)))
        if prolongations is not None:
            if len(prolongations) != h.levels_solver - 1:
                raise ValueError("prolongations needs levels_solver - 1 matrices, got %d"
                                 % len(prolongations))
            self._P = []
            self._P_c = (_capi.Csr * len(prolongations))()
            for k, Pm in enumerate(prolongations):
                Pm = Pm.tocsr()
                arrs = (np.ascontiguousarray(Pm.indptr, dtype=np.int64),
                        np.ascontiguousarray(Pm.indices, dtype=np.int32),
                        np.ascontiguousarray(Pm.data, dtype=np.float64))
                self._P.append(arrs)
                c = self._P_c[k]
                c.rows, c.cols = Pm.shape
                c.row_ptr = arrs[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                c.col_idx = arrs[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
                c.vals = arrs[2].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            h.P = ctypes.cast(self._P_c, ctypes.POINTER(_capi.Csr))
        o = default_options()
        self._weights = None
        for k, v in options.items():
            if k == "precision":
                v = PRECISIONS[v] if isinstance(v, str) else int(v)
            elif k == "alloc":
                v = ALLOCS[v] if isinstance(v, str) else int(v)
            elif k == "rho_weights":
                self._weights = np.ascontiguousarray(v, dtype=np.float64)
                o.rho_weights = self._weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                continue
            if not hasattr(o, k):
                raise TypeError("unknown option %r" % k)
            setattr(o, k, v)
        self.options = o
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        _check(self._lib.mlmc_setup(ctypes.byref(op), ctypes.byref(h), ctypes.byref(o),
                                    ctypes.c_void_p(stream.cuda_stream),
                                    ctypes.byref(self._ctx)), None)
        if not _exit_hook:
            # registered after torch is imported, so it runs before torch's own
            # exit handlers
            atexit.register(_close_live)
            _exit_hook.append(True)
        _live.add(self)
        self.kind = kind
        self.general = prolongations is not None  # general decomposition (given P)
        self.is_complex = kind in ("wilson2d", "gauge2d")
        self.levels_solver = h.levels_solver
        self.levels_mlmc = h.levels_mlmc
        self.nb = o.nb

    # -- lifetime --
    def close(self):
        if self._ctx:
            self._lib.mlmc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the allocator callbacks (and this module's
        # globals) may already be gone; the exit handler has closed every
        # estimator by then
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _c(self, rc):
        _check(rc, self._ctx)

    # -- estimator --
    def trace(self, tol, seed):
        r = _capi.Result()
        self._c(self._lib.mlmc_trace(self._ctx, float(tol), int(seed), ctypes.byref(r)))
        return _result_dict(r)

    def hutchinson(self, tol, seed):
        r = _capi.Result()
        self._c(self._lib.mlmc_hutchinson(self._ctx, float(tol), int(seed), ctypes.byref(r)))
        return _result_dict(r)

    # -- deflated Hutchinson (Sec. 4.2 / Sec. 5 comparison method) --
    def deflation_setup(self, n_defl, *, oversample=0, eig_tol=1e-3, max_iter=60,
                        solve_tol=1e-8, seed=1):
        """Eigenpairs of the n_defl smallest eigenvalues (subspace iteration on the
        library's solves) and the direct term tr(U^T A^-1 U); returns the report."""
        o = _capi.DeflationOptions(int(n_defl), int(oversample), float(eig_tol), int(max_iter),
                                   float(solve_tol), int(seed))
        r = _capi.DeflationReport()
        self._c(self._lib.mlmc_deflation_setup(self._ctx, ctypes.byref(o), ctypes.byref(r)))
        return dict(iterations=r.iterations, seconds=r.seconds, max_residual=r.max_residual,
                    direct_trace=r.direct_trace, sum_inv_eig=r.sum_inv_eig, solves=r.solves)

    def deflated_sample(self, seed, first, count, with_error=False):
        out = np.zeros((count, 2))
        err = np.zeros(count)
        self._c(self._lib.mlmc_deflated_sample(
            self._ctx, int(seed), int(first), int(count),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            err.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        s = out[:, 0] + 1j * out[:, 1]
        return (s, err) if with_error else s

    def deflated_hutchinson(self, tol, seed):
        r = _capi.Result()
        self._c(self._lib.mlmc_deflated_hutchinson(self._ctx, float(tol), int(seed),
                                                   ctypes.byref(r)))
        return _result_dict(r)

    def deflation_export(self, n_defl):
        """(eigenvalues [k], U [k, n_1] device tensor, direct term)."""
        import torch
        lam = np.zeros(int(n_defl))
        U = torch.empty((int(n_defl), self.level_size(1)), dtype=torch.float64, device="cuda")
        d = ctypes.c_double()
        self._c(self._lib.mlmc_deflation_export(
            self._ctx, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._ptr(U),
            ctypes.byref(d)))
        return lam, U, d.value

    def sample_level(self, level, seed, first, count, with_error=False):
        out = np.zeros((count, 2))
        err = np.zeros(count)
        self._c(self._lib.mlmc_sample_level(
            self._ctx, int(level), int(seed), int(first), int(count),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            err.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        s = out[:, 0] + 1j * out[:, 1]
        return (s, err) if with_error else s

    def coarse_trace(self):
        out = np.zeros(2)
        self._c(self._lib.mlmc_coarse_trace(self._ctx,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return complex(out[0], out[1])

    def level_size(self, level):
        n = ctypes.c_int64()
        self._c(self._lib.mlmc_level_size(self._ctx, int(level), ctypes.byref(n)))
        return n.value

    def counters(self):
        out = (ctypes.c_int64 * 4)()
        self._c(self._lib.mlmc_counters(self._ctx, out, 4))
        return list(out)

    # -- measurement --
    KERNELS = ["rbgs_sweep", "residual_restrict", "prolong_correct", "update_apply", "cg_xr",
               "nn_apply", "ir_fold", "ir_residual"]

    def set_timing(self, kernels=True, stride=1):
        """kernels: True (all), False (none) or a list of kernel names to time;
        stride: time every stride-th launch of each timed kernel."""
        if kernels is True:
            mask = (1 << len(self.KERNELS)) - 1
        elif not kernels:
            mask = 0
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << self.KERNELS.index(k)
        self._c(self._lib.mlmc_set_timing(self._ctx, int(mask), int(stride)))

    def reset_kernel_stats(self):
        self._c(self._lib.mlmc_reset_kernel_stats(self._ctx))

    def kernel_stats(self, kernel, fp64=False, level=0):
        """(launches, total ms, total algorithmic bytes) of a timed kernel, over all
        levels (level 0) or on one level."""
        kid = self.KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
        out = np.zeros(3)
        self._c(self._lib.mlmc_kernel_stats_level(
            self._ctx, kid, 1 if fp64 else 0, int(level),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return int(out[0]), float(out[1]), float(out[2])

    # -- FP64 building blocks on torch device tensors --
    def _vec(self, level, nrhs, device=None):
        import torch
        n = self.level_size(level)
        cols = 2 * n if self.is_complex else n
        return torch.empty((nrhs, cols), dtype=torch.float64, device=device or "cuda")

    @staticmethod
    def _ptr(t):
        import torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def _sync(self):
        self._stream.synchronize()

    def solve(self, level, b):
        """y = A_level^{-1} b for b [nrhs, n] (complex: [nrhs, 2n] interleaved)."""
        y = self._vec(level, b.shape[0], b.device)
        rel = np.zeros(b.shape[0])
        self._c(self._lib.mlmc_solve(self._ctx, int(level), int(b.shape[0]), self._ptr(b),
                                     self._ptr(y),
                                     rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return y, rel

    def apply(self, level, x):
        y = self._vec(level, x.shape[0], x.device)
        self._c(self._lib.mlmc_apply(self._ctx, int(level), int(x.shape[0]), self._ptr(x),
                                     self._ptr(y)))
        return y

    def smooth(self, level, b, x, sweeps, reverse=False, restrict=False, zero_start=False,
               noalloc=False, schedule=None):
        """`sweeps` red-black Gauss-Seidel sweeps of A_level x = b, in the working
        precision with the V-cycle's own kernels; returns the new x (x is not
        changed; with zero_start=True x may be None and the sweeps start from 0 with
        the pre-smoothing's zero-start kernels), and with restrict=True also
        R (b - A x) of it, as the V-cycle's last pre-smoothing pass forms it.
        reverse: second colour first, as in post-smoothing.  noalloc: through
        mlmc_smooth_noalloc (working copies in the library's fixed workspace).
        schedule (CSR kind): None the level's tuned sweep schedule, "classes" a
        launch per colour class, "shared_tail" the small trailing classes in
        shared launches."""
        import torch
        y = torch.empty_like(b) if x is None else x.clone()
        rc = self._vec(level + 1, b.shape[0], b.device) if restrict else None
        sched = {None: 0, "classes": _capi.SMOOTH_CLASS_LAUNCHES,
                 "shared_tail": _capi.SMOOTH_SHARED_TAIL}[schedule]
        flags = (_capi.SMOOTH_REVERSE if reverse else 0) | \
            (_capi.SMOOTH_ZERO_START if zero_start else 0) | sched
        fn = self._lib.mlmc_smooth_noalloc if noalloc else self._lib.mlmc_smooth
        self._c(fn(self._ctx, int(level), int(b.shape[0]), int(sweeps), flags, self._ptr(b),
                   self._ptr(y), self._ptr(rc) if restrict else None))
        if noalloc:
            self._sync()
        return (y, rc) if restrict else y

    def restrict(self, level, x):
        y = self._vec(level + 1, x.shape[0], x.device)
        self._c(self._lib.mlmc_restrict(self._ctx, int(level), int(x.shape[0]), self._ptr(x),
                                        self._ptr(y)))
        return y

    def prolong(self, level, xc):
        y = self._vec(level, xc.shape[0], xc.device)
        self._c(self._lib.mlmc_prolong(self._ctx, int(level), int(xc.shape[0]),
                                       self._ptr(xc), self._ptr(y)))
        return y

    def probes(self, level, seed, first, nrhs, stream=0):
        y = self._vec(level, nrhs)
        self._c(self._lib.mlmc_probes(self._ctx, int(level), int(seed), int(stream),
                                      int(first), int(nrhs), self._ptr(y)))
        return y

    def export_level(self, level, which="A"):
        """A_l (which="A") or P_l (which="P") as a scipy.sparse CSR matrix."""
        import scipy.sparse as sp
        w = 0 if which == "A" else 1
        rows, cols, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._c(self._lib.mlmc_export_level(self._ctx, int(level), w, ctypes.byref(rows),
                                            ctypes.byref(cols), ctypes.byref(nnz), None, None,
                                            None))
        rp = np.zeros(rows.value + 1, dtype=np.int64)
        ci = np.zeros(nnz.value, dtype=np.int32)
        v = np.zeros(nnz.value * (2 if self.is_complex else 1))
        self._c(self._lib.mlmc_export_level(
            self._ctx, int(level), w, None, None, None,
            rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        if self.is_complex:
            v = v[0::2] + 1j * v[1::2]
        return sp.csr_matrix((v, ci, rp), shape=(rows.value, cols.value))

    def export_csr(self, level):
        """Level `level` of a csr hierarchy: (scipy CSR matrix A_level, aggregate
        map, or None on the coarsest level and with given prolongations, colour
        classes)."""
        import scipy.sparse as sp
        n = self.level_size(level)
        nnz = ctypes.c_int64()
        self._c(self._lib.mlmc_export_csr(self._ctx, int(level), ctypes.byref(nnz), None, None,
                                          None, None, None))
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(nnz.value, dtype=np.int32)
        v = np.zeros(nnz.value)
        col = np.zeros(n, dtype=np.int32)
        agg = (np.zeros(n, dtype=np.int32)
               if level < self.levels_solver and not self.general else None)
        i32 = ctypes.POINTER(ctypes.c_int32)
        self._c(self._lib.mlmc_export_csr(
            self._ctx, int(level), ctypes.byref(nnz),
            rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ci.ctypes.data_as(i32),
            v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            agg.ctypes.data_as(i32) if agg is not None else None, col.ctypes.data_as(i32)))
        return sp.csr_matrix((v, ci, rp), shape=(n, n)), agg, col

    def export_coarse(self, which=0):
        lvl = self.levels_mlmc if which == 1 else self.levels_solver
        n = self.level_size(lvl)
        out = np.zeros((n, 2 * n) if self.is_complex else (n, n))
        self._c(self._lib.mlmc_export_coarse(self._ctx, int(which),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        if self.is_complex:
            out = out[:, 0::2] + 1j * out[:, 1::2]
        return out

    def export_prolongation(self, level, n_vec):
        n = self.level_size(level)
        out = np.zeros((n, 2 * n_vec))
        self._c(self._lib.mlmc_export_prolongation(
            self._ctx, int(level), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out[:, 0::2] + 1j * out[:, 1::2]

    # -- learned smoother (wilson2d) --
    def learned_train(self, w_init, *, n_batches=8, crops_per_column=4, steps=500, batch=256,
                      lr=1e-3, seed=1, pair_tol=0.0):
        """Train the network on (residual, error) pairs from the plain solver;
        returns the training report as a dict."""
        w = np.ascontiguousarray(w_init, dtype=np.float32)
        if w.size != _capi.NN_WEIGHTS:
            raise ValueError("w_init must hold %d weights" % _capi.NN_WEIGHTS)
        o = _capi.TrainOptions()
        o.n_batches, o.crops_per_column = int(n_batches), int(crops_per_column)
        o.steps, o.batch, o.lr, o.seed = int(steps), int(batch), float(lr), int(seed)
        o.pair_tol = float(pair_tol)
        rep = _capi.TrainReport()
        self._c(self._lib.mlmc_learned_train(
            self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(o),
            ctypes.byref(rep)))
        return {k: getattr(rep, k) for k, _ in _capi.TrainReport._fields_}

    def set_nn_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != _capi.NN_WEIGHTS:
            raise ValueError("weights must hold %d values" % _capi.NN_WEIGHTS)
        self._c(self._lib.mlmc_learned_set_weights(
            self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_nn_weights(self):
        w = np.zeros(_capi.NN_WEIGHTS, dtype=np.float32)
        self._c(self._lib.mlmc_learned_get_weights(
            self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return w

    def learned_stats(self):
        """(network applications, fallbacks to the plain smoother) since setup."""
        out = (ctypes.c_int64 * 2)()
        self._c(self._lib.mlmc_learned_stats(self._ctx, out))
        return int(out[0]), int(out[1])

    def nn_apply(self, r):
        """Correction of the network for residuals r [nrhs, 2 n_1] (interleaved
        complex FP64 on the device)."""
        e = self._vec(1, r.shape[0], r.device)
        self._c(self._lib.mlmc_nn_apply(self._ctx, int(r.shape[0]), self._ptr(r), self._ptr(e)))
        return e

    def nn_loss_grad(self, inputs, targets):
        """Mean squared error and weight gradient over crops: inputs [B, 22, 22, 8]
        and targets [B, 16, 16, 4], FP32 device tensors."""
        import torch
        assert inputs.dtype == torch.float32 and targets.dtype == torch.float32
        assert tuple(inputs.shape[1:]) == (22, 22, 8) and tuple(targets.shape[1:]) == (16, 16, 4)
        assert inputs.is_cuda and targets.is_cuda
        assert inputs.is_contiguous() and targets.is_contiguous()
        loss = ctypes.c_double()
        grad = np.zeros(_capi.NN_WEIGHTS, dtype=np.float32)
        self._c(self._lib.mlmc_nn_loss_grad(
            self._ctx, int(inputs.shape[0]), ctypes.c_void_p(inputs.data_ptr()),
            ctypes.c_void_p(targets.data_ptr()),
            ctypes.byref(loss), grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return loss.value, grad

    def nn_crops(self, r, e, origins):
        """Training crops from residuals r and errors e (device FP64 complex-interleaved
        [nrhs, 2 n_1]) at origins [ncrops, 3] = (column, y0, x0): (inputs
        [ncrops, 22, 22, 8], targets [ncrops, 16, 16, 4]) as FP32 host arrays."""
        assert tuple(r.shape) == tuple(e.shape) and r.shape[1] == 2 * self.level_size(1)
        nrhs = int(r.shape[0])
        org = np.ascontiguousarray(origins, dtype=np.int32)
        nc = int(org.shape[0])
        inp = np.zeros((nc, 22, 22, 8), dtype=np.float32)
        tgt = np.zeros((nc, 16, 16, 4), dtype=np.float32)
        self._c(self._lib.mlmc_nn_crops(
            self._ctx, nrhs, self._ptr(r), self._ptr(e), nc,
            org.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            inp.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            tgt.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return inp, tgt

    def nn_adam_step(self, grad, lr, t):
        """One Adam update of the network's master weights with gradient grad."""
        g = np.ascontiguousarray(grad, dtype=np.float32)
        assert g.size == _capi.NN_WEIGHTS
        self._c(self._lib.mlmc_nn_adam_step(
            self._ctx, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), float(lr), int(t)))


def batch_sample(estimators, level, seeds, first, nsamples, workers=4):
    """Samples of one level on several problems at once (mlmc_batch_sample).
    Returns (samples [count, nsamples] complex, seconds per problem)."""
    count = len(estimators)
    ctxs = (ctypes.c_void_p * count)(*[e._ctx.value for e in estimators])
    sd = (ctypes.c_uint64 * count)(*[int(v) for v in seeds])
    out = np.zeros((count, int(nsamples), 2))
    sec = np.zeros(count)
    rc = lib().mlmc_batch_sample(ctxs, count, int(level), sd, int(first), int(nsamples),
                                 int(workers), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 sec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        msgs = [e._lib.mlmc_last_error(e._ctx) for e in estimators]
        msg = next((m.decode() for m in msgs if m), "")
        raise MLMCError(rc, msg)
    return out[..., 0] + 1j * out[..., 1], sec


def stream_copy(src, dst):
    """Device copy src -> dst (torch tensors of equal byte size, multiple of 16)
    with the library's streaming kernel on torch's current stream."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = torch.cuda.current_stream().cuda_stream
    rc = lib().mlmc_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                nbytes, ctypes.c_void_p(s))
    if rc != 0:
        raise MLMCError(rc, "stream copy")


def batch_sample_grouped(estimators, level, seeds, first, nsamples, persistent=False):
    """Samples of one level on several problems solved in lockstep on one stream
    (mlmc_batch_sample_grouped): persistent=True runs each V-cycle of all problems
    as one persistent launch (a workgroup per problem and column pair), False as
    one launch per stage position.  Returns (samples [count, nsamples] complex,
    status per problem)."""
    count = len(estimators)
    ctxs = (ctypes.c_void_p * count)(*[e._ctx.value for e in estimators])
    sd = (ctypes.c_uint64 * count)(*[int(v) for v in seeds])
    out = np.zeros((count, int(nsamples), 2))
    st = (ctypes.c_int * count)()
    rc = lib().mlmc_batch_sample_grouped(ctxs, count, int(level), sd, int(first), int(nsamples),
                                         1 if persistent else 2,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), st)
    if rc != 0:
        msgs = [e._lib.mlmc_last_error(e._ctx) for e in estimators]
        msg = next((m.decode() for m in msgs if m), "")
        raise MLMCError(rc, msg)
    return out[..., 0] + 1j * out[..., 1], list(st)


def run_estimator(levels, sample, tol, *, pilot=None, coarse=0.0, cost=None, **options):
    """Host-side estimator over a Python sampler (no device use).

    sample(level, first, count) -> complex array; pilot(count) -> complex array.
    """
    L = lib()
    o = default_options()
    weights = None
    for k, v in options.items():
        if k == "alloc":
            v = ALLOCS[v] if isinstance(v, str) else int(v)
        if k == "rho_weights":
            weights = np.ascontiguousarray(v, dtype=np.float64)
            o.rho_weights = weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            continue
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    errors = []

    def _fill(vals, count, out):
        vals = np.asarray(vals, dtype=np.complex128)
        assert vals.shape == (count,)
        for i in range(count):
            out[2 * i] = vals[i].real
            out[2 * i + 1] = vals[i].imag

    def _sample(_user, level, first, count, out):
        try:
            _fill(sample(level, first, count), count, out)
            return 0
        except Exception as e:  # reported through the status code
            errors.append(e)
            return -1

    def _pilot(_user, count, out):
        try:
            _fill(pilot(count), count, out)
            return 0
        except Exception as e:
            errors.append(e)
            return -1

    sf = _capi.SAMPLE_FN(_sample)
    pf = _capi.PILOT_FN(_pilot) if pilot is not None else _capi.PILOT_FN(0)
    cz = np.array([complex(coarse).real, complex(coarse).imag])
    cv = None if cost is None else np.ascontiguousarray(cost, dtype=np.float64)
    r = _capi.Result()
    rc = L.mlmc_run_estimator(
        int(levels), sf, pf, None, cz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        None if cv is None else cv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        ctypes.byref(o), float(tol), ctypes.byref(r))
    if errors:
        raise errors[0]
    _check(rc)
    return _result_dict(r)
