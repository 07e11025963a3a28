"""Python binding of libmlc.so (include/mlc.h): argument marshalling only.

Every computation happens inside the library's HIP kernels and host C++ code.
PyTorch supplies the device workspace and the HIP stream. If the shared
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libmlc.so"
_lib = None

MLC_OK = 0
MLC_WARN_INNER_MAXIT = 1
STATUS = {0: "MLC_OK", -1: "MLC_ERR_ARG", -2: "MLC_ERR_MESH", -3: "MLC_ERR_NOT_NESTED", -4: "MLC_ERR_WORKSPACE",
          -5: "MLC_ERR_HIP", -6: "MLC_ERR_NOT_CONVERGED", -7: "MLC_ERR_BREAKDOWN", -8: "MLC_ERR_NONFINITE",
          -9: "MLC_ERR_STATE", 1: "MLC_WARN_INNER_MAXIT"}

PROBES = ["U", "W0", "G", "VXC_QP", "PT_AFIX_U", "PT_MW0_U", "PT_M_U", "PT_K_U", "UT_AFIX_U", "UT_MW0_U",
          "UT_M_U", "UT_K_U", "HARTREE_D", "AFIX_H", "MW0_H", "M_H", "K_H", "AH4", "RHS", "THETA2", "PHI_H",
          "WH", "SIGMA", "FEATURES", "NN_OUT", "GUESS_SCALE", "PATTERN", "LMAX"]
PROBE_ID = {name: i for i, name in enumerate(PROBES)}

EXPORTED = ["mlc_options_default", "mlc_create", "mlc_sizes", "mlc_workspace_bytes", "mlc_bind",
            "mlc_initial_state", "mlc_set_state", "mlc_correction_step", "mlc_get_results", "mlc_probe",
            "mlc_time_kernel", "mlc_status_string", "mlc_last_error", "mlc_destroy", "mlc_batch_create",
            "mlc_batch_workspace_bytes", "mlc_batch_bind", "mlc_batch_set_shape", "mlc_batch_step",
            "mlc_batch_last_error", "mlc_batch_destroy", "mlc_nn_create", "mlc_nn_workspace_bytes", "mlc_nn_bind",
            "mlc_nn_set_params", "mlc_nn_get_params", "mlc_nn_forward", "mlc_nn_loss_grad", "mlc_nn_adam",
            "mlc_nn_train", "mlc_nn_last_error", "mlc_nn_destroy", "mlc_set_guess", "mlc_set_sample_sink",
            "mlc_sample_count", "mlc_nn_loss_grad_noalloc", "mlc_estimate", "mlc_mark_dorfler", "mlc_refine",
            "mlc_refine_free", "mlc_transfer_vertices"]
N_PARAMS = 8833


class MlcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("order", C.c_int32), ("n_vertices", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("n_tets", C.c_int64),
                ("tets", C.POINTER(C.c_int32))]


class SystemDesc(C.Structure):
    _fields_ = [("n_nuclei", C.c_int32), ("R", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_double)),
                ("potential", C.c_int32), ("rc", C.c_double), ("omega", C.c_double), ("n_orbitals", C.c_int32),
                ("occupations", C.POINTER(C.c_double)), ("xc", C.c_int32), ("xalpha", C.c_double),
                ("hartree", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3)]


class Options(C.Structure):
    _fields_ = [("cg_rtol", C.c_double), ("cg_maxit", C.c_int32), ("check_every", C.c_int32),
                ("shift", C.c_int32), ("sigma0", C.c_double), ("poisson_rtol", C.c_double),
                ("inner_maxit", C.c_int32), ("inner_tol", C.c_double), ("n_extra", C.c_int32),
                ("reorder", C.c_int32), ("time_kernels", C.c_int32), ("use_graphs", C.c_int32),
                ("precision", C.c_int32), ("ir_inner_rtol", C.c_double), ("ir_max_outer", C.c_int32),
                ("precond", C.c_int32), ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
                ("hartree_coarse", C.c_int32), ("hartree_precond", C.c_int32),
                ("inner_mix_history", C.c_int32), ("inner_mix_beta", C.c_double), ("variant", C.c_int32),
                ("estimator", C.c_int32), ("cheb_lanczos", C.c_int32),
                ("hartree_cheb_degree", C.c_int32), ("hartree_cheb_ratio", C.c_double)]

PREC_FP64, PREC_FP32_IR = 0, 1
PC_JACOBI, PC_CHEBYSHEV = 0, 1
VARIANT_EIGENPAIRWISE, VARIANT_JOINT = 0, 1
KERNELS = {"cg_spmm": 0, "cheb_step": 1, "hartree_spmm": 2, "hartree_cheb_step": 3}


class StepReport(C.Structure):
    _fields_ = [("cg_iters_max", C.c_int32), ("cg_iters_sum", C.c_int32), ("poisson_iters", C.c_int32),
                ("inner_iters", C.c_int32), ("cg_relres_max", C.c_double), ("poisson_relres", C.c_double),
                ("inner_last_diff", C.c_double), ("sigma", C.c_double), ("theta1", C.c_double),
                ("max_offdiag_overlap", C.c_double), ("rho_integral", C.c_double), ("energy", C.c_double),
                ("t_fine_ms", C.c_double), ("t_inner_ms", C.c_double), ("t_recon_ms", C.c_double),
                ("t_spmm_ms", C.c_double), ("n_spmm", C.c_int64), ("spmm_rows", C.c_int64),
                ("spmm_cols_sum", C.c_int64), ("ir_outer", C.c_int32), ("guess_learned_cols", C.c_int32),
                ("guess_resid_ratio", C.c_double), ("t_solve_ms", C.c_double), ("t_poisson_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchReport(C.Structure):
    _fields_ = [("n_systems", C.c_int32), ("tile_rows", C.c_int32), ("spmm_lanes", C.c_int32),
                ("n_tiles", C.c_int32), ("cg_iters", C.c_int32), ("poisson_iters", C.c_int32),
                ("ir_outer", C.c_int32), ("pad", C.c_int32), ("dof_orbitals", C.c_int64),
                ("t_gpu_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_poisson_ms", C.c_double),
                ("t_inner_ms", C.c_double), ("t_recon_ms", C.c_double), ("t_tune_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


class RefineResult(C.Structure):
    _fields_ = [("nv", C.c_int64), ("nt", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("tets", C.POINTER(C.c_int32)), ("tags", C.POINTER(C.c_int8)), ("n_new", C.c_int64),
                ("parents", C.POINTER(C.c_int64)), ("nbatch", C.c_int32), ("batch_ptr", C.POINTER(C.c_int64)),
                ("internal", C.c_void_p)]


def lib():
    """Load libmlc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2103_02824_amd.build`")
    L = C.CDLL(str(LIB_PATH))
    P, i32, i64, dbl, vp = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    L.mlc_options_default.argtypes = [P(Options)]
    L.mlc_options_default.restype = None
    L.mlc_create.argtypes = [P(Mesh), P(Mesh), P(SystemDesc), P(Options), P(vp)]
    L.mlc_sizes.argtypes = [vp, P(i64), P(i64), P(i64), P(i32)]
    L.mlc_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.mlc_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.mlc_initial_state.argtypes = [vp, dbl, i32, P(i32)]
    L.mlc_set_state.argtypes = [vp, P(dbl), P(dbl), P(dbl)]
    L.mlc_correction_step.argtypes = [vp, P(StepReport)]
    L.mlc_get_results.argtypes = [vp, P(dbl), P(dbl), P(dbl), P(dbl)]
    L.mlc_probe.argtypes = [vp, i32, P(dbl), i64]
    L.mlc_time_kernel.argtypes = [vp, i32, i32, P(dbl)]
    L.mlc_time_kernel.restype = i32
    L.mlc_estimate.argtypes = [vp, vp]
    L.mlc_estimate.restype = i32
    L.mlc_mark_dorfler.argtypes = [P(dbl), i64, dbl, P(C.c_uint8), P(i64)]
    L.mlc_mark_dorfler.restype = i32
    L.mlc_refine.argtypes = [i64, P(dbl), i64, P(i32), P(C.c_int8), P(C.c_uint8), P(RefineResult)]
    L.mlc_refine.restype = i32
    L.mlc_refine_free.argtypes = [P(RefineResult)]
    L.mlc_refine_free.restype = None
    L.mlc_transfer_vertices.argtypes = [i64, i64, vp, i32, P(i64), i32, vp, vp]
    L.mlc_transfer_vertices.restype = i32
    L.mlc_status_string.argtypes = [i32]
    L.mlc_status_string.restype = C.c_char_p
    L.mlc_last_error.argtypes = [vp]
    L.mlc_last_error.restype = C.c_char_p
    L.mlc_destroy.argtypes = [vp]
    L.mlc_destroy.restype = None
    L.mlc_batch_create.argtypes = [P(vp), i32, P(vp)]
    L.mlc_batch_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.mlc_batch_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.mlc_batch_set_shape.argtypes = [vp, i32, i32]
    L.mlc_batch_step.argtypes = [vp, P(StepReport), P(BatchReport)]
    L.mlc_batch_last_error.argtypes = [vp]
    L.mlc_batch_last_error.restype = C.c_char_p
    L.mlc_batch_destroy.argtypes = [vp]
    L.mlc_batch_destroy.restype = None
    fp = P(C.c_float)
    L.mlc_nn_create.argtypes = [P(vp)]
    L.mlc_nn_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.mlc_nn_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.mlc_nn_set_params.argtypes = [vp, fp]
    L.mlc_nn_get_params.argtypes = [vp, fp]
    L.mlc_nn_forward.argtypes = [vp, vp, i64, vp]
    L.mlc_nn_loss_grad.argtypes = [vp, vp, vp, i64, P(dbl), fp]
    L.mlc_nn_adam.argtypes = [vp, fp, dbl, dbl, dbl, dbl]
    L.mlc_nn_loss_grad_noalloc.argtypes = [vp, vp, vp, i64, P(dbl), fp]
    L.mlc_nn_loss_grad_noalloc.restype = i32
    L.mlc_nn_train.argtypes = [vp, vp, vp, i64, i32, i32, dbl, fp]
    L.mlc_nn_last_error.argtypes = [vp]
    L.mlc_nn_last_error.restype = C.c_char_p
    L.mlc_nn_destroy.argtypes = [vp]
    L.mlc_nn_destroy.restype = None
    L.mlc_set_guess.argtypes = [vp, vp]
    L.mlc_set_sample_sink.argtypes = [vp, vp, vp, i64, i32]
    L.mlc_sample_count.argtypes = [vp, P(i64)]
    for f in ("mlc_nn_create", "mlc_nn_workspace_bytes", "mlc_nn_bind", "mlc_nn_set_params", "mlc_nn_get_params",
              "mlc_nn_forward", "mlc_nn_loss_grad", "mlc_nn_adam", "mlc_nn_train", "mlc_set_guess",
              "mlc_set_sample_sink", "mlc_sample_count"):
        getattr(L, f).restype = i32
    for f in ("mlc_batch_create", "mlc_batch_workspace_bytes", "mlc_batch_bind", "mlc_batch_set_shape",
              "mlc_batch_step"):
        getattr(L, f).restype = i32
    for f in ("mlc_create", "mlc_sizes", "mlc_workspace_bytes", "mlc_bind", "mlc_initial_state", "mlc_set_state",
              "mlc_correction_step", "mlc_get_results", "mlc_probe"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def box3(v):
    """A box bound as the C double[3]: a scalar for all three axes, or three values."""
    a = np.broadcast_to(np.asarray(v, dtype=np.float64), (3,))
    return (C.c_double * 3)(*[float(x) for x in a])


def options(**kw):
    o = Options()
    lib().mlc_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Context:
    """One library context bound to a torch-allocated workspace and stream."""

    def __init__(self, system, opts: Options = None, device="cuda:0"):
        import torch

        L = lib()
        self._keep = []
        xyz = np.ascontiguousarray(system.xyz, dtype=np.float64)
        tets = np.ascontiguousarray(system.tets, dtype=np.int32)
        cxyz = np.ascontiguousarray(system.cxyz, dtype=np.float64)
        ctets = np.ascontiguousarray(system.ctets, dtype=np.int32)
        R = np.ascontiguousarray(np.asarray(system.R, dtype=np.float64).reshape(-1, 3))
        Z = np.ascontiguousarray(np.asarray(system.Z, dtype=np.float64).ravel())
        occ = np.ascontiguousarray(np.asarray(system.occupations, dtype=np.float64))
        self._keep += [xyz, tets, cxyz, ctets, R, Z, occ]
        order = int(getattr(system, "order", 1))
        fine = Mesh(order, len(xyz), _dp(xyz), len(tets), tets.ctypes.data_as(C.POINTER(C.c_int32)))
        coarse = Mesh(1, len(cxyz), _dp(cxyz), len(ctets), ctets.ctypes.data_as(C.POINTER(C.c_int32)))
        sd = SystemDesc(len(Z), _dp(R), _dp(Z), int(system.potential), float(system.rc), float(system.omega),
                        int(system.n_orbitals), _dp(occ), int(system.xc), float(system.xalpha),
                        int(bool(system.hartree)), box3(system.lo), box3(system.hi))
        self.opts = opts if opts is not None else options()
        h = C.c_void_p()
        st = L.mlc_create(C.byref(fine), C.byref(coarse), C.byref(sd), C.byref(self.opts), C.byref(h))
        if st != MLC_OK:
            msg = L.mlc_last_error(h).decode() if h.value else "mlc_create failed"
            if h.value:
                L.mlc_destroy(h)
            raise MlcError(st, msg)
        self.h = h
        n, nH, nv, N = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        self._chk(L.mlc_sizes(h, C.byref(n), C.byref(nH), C.byref(nv), C.byref(N)))
        self.n_dof, self.n_coarse_dof, self.n_vertices, self.N = n.value, nH.value, nv.value, N.value
        self.n_tets = len(tets)
        nbytes = C.c_size_t()
        self._chk(L.mlc_workspace_bytes(h, C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._chk(L.mlc_bind(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                             C.c_void_p(self.stream.cuda_stream)))

    def _chk(self, st, allow_warn=False):
        if st == MLC_OK or (allow_warn and st > 0):
            return st
        raise MlcError(st, lib().mlc_last_error(self.h).decode())

    def initial_state(self, tol=1e-11, maxit=400):
        it = C.c_int32()
        self._chk(lib().mlc_initial_state(self.h, tol, maxit, C.byref(it)))
        return it.value

    def _dev(self, a, shape):
        """a (NumPy array or torch tensor) as a contiguous float64 tensor of the given shape on the
        context's device."""
        import torch
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).reshape(shape).contiguous()
        return t

    def set_state(self, lam, Phi, w):
        """lam: host (N,); Phi (n_dof, N) and w (n_vertices,): NumPy arrays or device tensors
        (copied to the device first when they are on the host)."""
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        assert lam.shape == (self.N,)
        P = self._dev(Phi, (self.n_dof, self.N))
        wd = self._dev(w, (self.n_vertices,))
        self._chk(lib().mlc_set_state(self.h, _dp(lam), C.cast(C.c_void_p(P.data_ptr()), C.POINTER(C.c_double)),
                                      C.cast(C.c_void_p(wd.data_ptr()), C.POINTER(C.c_double))))

    def correction_step(self, allow_warn=True):
        rep = StepReport()
        st = lib().mlc_correction_step(self.h, C.byref(rep))
        self._chk(st, allow_warn=allow_warn)
        d = rep.as_dict()
        d["status"] = st
        return d

    def get_results_device(self):
        """(lam host NumPy (N,), Phi (n_dof, N), w (n_vertices,), rho (n_vertices,) as device tensors)."""
        import torch
        lam = np.zeros(self.N)
        Phi = torch.empty((self.n_dof, self.N), dtype=torch.float64, device=self.device)
        w = torch.empty(self.n_vertices, dtype=torch.float64, device=self.device)
        rho = torch.empty(self.n_vertices, dtype=torch.float64, device=self.device)
        dp = lambda t: C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_double))
        self._chk(lib().mlc_get_results(self.h, _dp(lam), dp(Phi), dp(rho), dp(w)))
        return lam, Phi, w, rho

    def get_results(self):
        """(lam, Phi, w, rho) as host NumPy arrays (copied from the device tensors)."""
        lam, Phi, w, rho = self.get_results_device()
        return lam, Phi.cpu().numpy(), w.cpu().numpy(), rho.cpu().numpy()

    def probe(self, name, shape):
        out = np.zeros(int(np.prod(shape)))
        self._chk(lib().mlc_probe(self.h, PROBE_ID[name], _dp(out), out.size))
        return out.reshape(shape)

    def set_guess(self, nn):
        """Start step 5 from the network's guess (None: from phi)."""
        self._chk(lib().mlc_set_guess(self.h, nn.h if nn is not None else None))
        self._guess = nn

    def set_sample_sink(self, x, t, stride=1):
        """x: torch float32 (capacity, 6), t: torch float32 (capacity,) on the device; None switches off."""
        if x is None:
            self._chk(lib().mlc_set_sample_sink(self.h, None, None, 0, 1))
            self._sink = None
            return
        assert x.dtype == t.dtype and x.shape[1] == 6 and x.shape[0] == t.shape[0] and x.is_contiguous()
        self._sink = (x, t)
        self._chk(lib().mlc_set_sample_sink(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                            int(x.shape[0]), int(stride)))

    def sample_count(self):
        r = C.c_int64()
        self._chk(lib().mlc_sample_count(self.h, C.byref(r)))
        return r.value

    def estimate(self):
        """eta^2 of the current state per fine tet (the residual estimator of
        the adaptive loop), a device tensor in the caller's tet order; needs
        options(estimator=1)."""
        import torch
        eta2 = torch.empty(self.n_tets, dtype=torch.float64, device=self.device)
        self._chk(lib().mlc_estimate(self.h, C.c_void_p(eta2.data_ptr())))
        return eta2

    def time_kernel(self, which="cg_spmm", reps=50):
        """Mean launch time (us) of one solver kernel replayed back to back:
        cg_spmm, cheb_step, hartree_spmm, hartree_cheb_step."""
        us = C.c_double()
        self._chk(lib().mlc_time_kernel(self.h, KERNELS[which], int(reps), C.byref(us)))
        return us.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mlc_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mark_dorfler(eta2, theta):
    """Doerfler set of eta2 (host array): (boolean mask, count)."""
    e = np.ascontiguousarray(eta2, dtype=np.float64)
    m = np.zeros(len(e), dtype=np.uint8)
    k = C.c_int64()
    st = lib().mlc_mark_dorfler(_dp(e), len(e), float(theta), m.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(k))
    if st != MLC_OK:
        raise MlcError(st, "mlc_mark_dorfler")
    return m.astype(bool), k.value


def refine(xyz, tets, tags, marked):
    """Bisect the marked tets and close the mesh (mlc_refine). Returns a dict
    of NumPy copies: xyz, tets, tags, parents (n_new x 2) and batch_ptr."""
    X = np.ascontiguousarray(xyz, dtype=np.float64)
    T = np.ascontiguousarray(tets, dtype=np.int32)
    G = np.ascontiguousarray(tags, dtype=np.int8)
    M = np.ascontiguousarray(marked, dtype=np.uint8)
    r = RefineResult()
    st = lib().mlc_refine(len(X), _dp(X), len(T), T.ctypes.data_as(C.POINTER(C.c_int32)),
                          G.ctypes.data_as(C.POINTER(C.c_int8)), M.ctypes.data_as(C.POINTER(C.c_uint8)),
                          C.byref(r))
    if st != MLC_OK:
        raise MlcError(st, "mlc_refine")
    try:
        out = {"xyz": np.ctypeslib.as_array(r.xyz, shape=(r.nv, 3)).copy(),
               "tets": np.ctypeslib.as_array(r.tets, shape=(r.nt, 4)).copy(),
               "tags": np.ctypeslib.as_array(r.tags, shape=(r.nt,)).copy(),
               "parents": (np.ctypeslib.as_array(r.parents, shape=(r.n_new, 2)).copy() if r.n_new
                           else np.zeros((0, 2), dtype=np.int64)),
               "batch_ptr": np.ctypeslib.as_array(r.batch_ptr, shape=(r.nbatch + 1,)).copy()}
    finally:
        lib().mlc_refine_free(C.byref(r))
    return out


def transfer_vertices(values, nv_old, parents, batch_ptr, stream=None):
    """Fill the new vertices' rows of values (device tensor, nv_new x ncols,
    float64, the first nv_old rows holding the old values) with the means of
    their parents' rows, batch by batch (mlc_transfer_vertices)."""
    import torch
    assert values.dtype == torch.float64 and values.is_contiguous()
    v2 = values.reshape(values.shape[0], -1)
    par = torch.as_tensor(np.ascontiguousarray(parents, dtype=np.int64).reshape(-1), device=values.device)
    bp = np.ascontiguousarray(batch_ptr, dtype=np.int64)
    s = stream if stream is not None else torch.cuda.current_stream(values.device)
    st = lib().mlc_transfer_vertices(int(nv_old), int(v2.shape[0]), C.c_void_p(par.data_ptr()), len(bp) - 1,
                                     bp.ctypes.data_as(C.POINTER(C.c_int64)), int(v2.shape[1]),
                                     C.c_void_p(v2.data_ptr()), C.c_void_p(s.cuda_stream))
    if st != MLC_OK:
        raise MlcError(st, "mlc_transfer_vertices")
    s.synchronize()  # keeps par alive until the kernels have read it
    return values


class Batch:
    """Several contexts stepped together (mlc_batch_*): batched CG launches for
    the step-5 and Hartree solves of every system, on one stream."""

    def __init__(self, contexts, tile_rows=0, lanes=0):
        import torch

        L = lib()
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        st = L.mlc_batch_create(arr, len(self.contexts), C.byref(h))
        if st != MLC_OK:
            raise MlcError(st, "mlc_batch_create failed")
        self.h = h
        nbytes = C.c_size_t()
        self._chk(L.mlc_batch_workspace_bytes(h, C.byref(nbytes)))
        dev = self.contexts[0].device
        self.workspace = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        self._chk(L.mlc_batch_bind(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                   C.c_void_p(self.stream.cuda_stream)))
        if tile_rows or lanes:
            self._chk(L.mlc_batch_set_shape(h, int(tile_rows), int(lanes)))

    def _chk(self, st, allow_warn=False):
        if st == MLC_OK or (allow_warn and st > 0):
            return st
        raise MlcError(st, lib().mlc_batch_last_error(self.h).decode())

    def step(self, allow_warn=True):
        reps = (StepReport * len(self.contexts))()
        br = BatchReport()
        st = lib().mlc_batch_step(self.h, reps, C.byref(br))
        self._chk(st, allow_warn=allow_warn)
        out = [r.as_dict() for r in reps]
        return out, br.as_dict()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mlc_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    """The learned-guess network (mlc_nn_*): parameters, forward, loss and
    gradient, Adam, training, all on the device through the library."""

    def __init__(self, device="cuda:0"):
        import torch

        L = lib()
        h = C.c_void_p()
        st = L.mlc_nn_create(C.byref(h))
        if st != MLC_OK:
            raise MlcError(st, "mlc_nn_create failed")
        self.h = h
        nbytes = C.c_size_t()
        self._chk(L.mlc_nn_workspace_bytes(h, C.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._chk(L.mlc_nn_bind(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                C.c_void_p(self.stream.cuda_stream)))

    def _chk(self, st):
        if st != MLC_OK:
            raise MlcError(st, lib().mlc_nn_last_error(self.h).decode())

    @staticmethod
    def _fp(a):
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == N_PARAMS
        self._chk(lib().mlc_nn_set_params(self.h, self._fp(th)))

    def get_params(self):
        th = np.zeros(N_PARAMS, dtype=np.float32)
        self._chk(lib().mlc_nn_get_params(self.h, self._fp(th)))
        return th

    def forward(self, x):
        """x: torch float32 (rows, 6) on the device -> torch float32 (rows,)."""
        import torch
        assert x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == 6
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._chk(lib().mlc_nn_forward(self.h, C.c_void_p(x.data_ptr()), int(x.shape[0]),
                                       C.c_void_p(y.data_ptr())))
        return y

    def loss_grad(self, x, t):
        g = np.zeros(N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        self._chk(lib().mlc_nn_loss_grad(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                         int(x.shape[0]), C.byref(loss), self._fp(g)))
        return loss.value, g

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        self._chk(lib().mlc_nn_adam(self.h, self._fp(g), lr, beta1, beta2, eps))

    def train(self, x, t, steps, batch=4096, lr=1e-3):
        hist = np.zeros(steps, dtype=np.float32)
        self._chk(lib().mlc_nn_train(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                     int(x.shape[0]), int(steps), int(batch), float(lr), self._fp(hist)))
        return hist

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().mlc_nn_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
