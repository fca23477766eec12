"""Thin ctypes binding of libclsel.so (include/clsel.h).

Argument marshalling only: every numeric step runs in the HIP library. Tensors are
torch tensors on the GPU (complex128, contiguous); the library is handed their
device pointers and torch's current HIP stream. If the library is missing, or no
GPU is usable, the numeric calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclsel.so")

CL_OK, CL_EINVAL, CL_ENOMEM, CL_EORDER = 0, -1, -2, -3
CL_ESINGULAR, CL_ENONFINITE, CL_EHIP, CL_ENODEV, CL_ERANK = -4, -5, -6, -7, -8
FRONT_FIELDS = ["id", "parent", "level", "npiv", "nstr", "p", "s", "H", "ld", "off", "site_off",
                "nchild", "child0", "child1", "child2", "child3", "inv_off0", "inv_off1",
                "inv_off2", "inv_off3", "rel_off", "nsteps", "fbuf", "zbuf", "r0", "r1", "r2", "r3"]


class ClselError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [("leaf_sites", ctypes.c_int32), ("max_pivot_rows", ctypes.c_int32),
                ("nb", ctypes.c_int32), ("time_cuts", ctypes.c_int32), ("gemm_tile", ctypes.c_int32),
                ("lowrank_cap", ctypes.c_int32), ("pivot_floor", ctypes.c_double),
                ("smw_refine", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("volume", ctypes.c_int64), ("n", ctypes.c_int64),
                ("nfronts", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("max_front_rows", ctypes.c_int32),
                ("max_pivot_rows", ctypes.c_int32), ("pool_elems", ctypes.c_int64),
                ("flops_factor", ctypes.c_double), ("flops_selinv", ctypes.c_double),
                ("flops_factor_alg", ctypes.c_double), ("flops_selinv_alg", ctypes.c_double),
                ("flops_dense_inverse", ctypes.c_double), ("lowrank_cap", ctypes.c_int32),
                ("pivot_floor", ctypes.c_double), ("smw_refine", ctypes.c_int32)]


_lib = None

EXPORTS = ["cl_symbolic", "cl_symbolic_ex", "cl_plan_info", "cl_plan_bytes", "cl_plan_export",
           "cl_plan_destroy", "cl_batch_create", "cl_batch_set_active", "cl_batch_use_graph",
           "cl_factor", "cl_selinv", "cl_drift", "cl_selected", "cl_run", "cl_status",
           "cl_batch_sync", "cl_batch_destroy", "cl_strerror", "cl_last_error",
           "cl_batch_profile", "cl_batch_profile_read", "cl_batch_profile_launches", "cl_batch_query", "cl_observables",
           "cl_gauge_drift", "cl_langevin_update", "cl_solve", "cl_stochastic_blocks",
           "cl_drift_from_blocks", "cl_batch_perturbations", "cl_run_noalloc", "cl_batch_inject_fault",
           "cl_batch_set_lanes"]


def lib():
    """Load libclsel.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ClselError(CL_ENODEV, f"{LIB_PATH} not built: run paper_1707_08874_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    sig = {
        "cl_symbolic": (ctypes.c_int, [i32p, ctypes.POINTER(vp)]),
        "cl_symbolic_ex": (ctypes.c_int, [i32p, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]),
        "cl_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(PlanInfo)]),
        "cl_plan_bytes": (ctypes.c_size_t, [vp, ctypes.c_int32]),
        "cl_plan_export": (ctypes.c_int, [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_size_t)]),
        "cl_plan_destroy": (None, [vp]),
        "cl_batch_create": (ctypes.c_int, [vp, ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "cl_batch_set_active": (ctypes.c_int, [vp, ctypes.c_int32]),
        "cl_batch_use_graph": (ctypes.c_int, [vp, ctypes.c_int32]),
        "cl_factor": (ctypes.c_int, [vp, vp, dp, dp]),
        "cl_selinv": (ctypes.c_int, [vp]),
        "cl_drift": (ctypes.c_int, [vp, vp]),
        "cl_selected": (ctypes.c_int, [vp, vp]),
        "cl_run": (ctypes.c_int, [vp, vp, dp, dp, vp, vp]),
        "cl_status": (ctypes.c_int, [vp, i32p]),
        "cl_batch_sync": (ctypes.c_int, [vp]),
        "cl_batch_destroy": (None, [vp]),
        "cl_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "cl_last_error": (ctypes.c_char_p, []),
        "cl_batch_profile": (ctypes.c_int, [vp, ctypes.c_int32]),
        "cl_batch_profile_read": (ctypes.c_int, [vp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "cl_batch_profile_launches": (ctypes.c_int, [vp, ctypes.c_int64, dp, dp, dp,
                                                      ctypes.POINTER(ctypes.c_int32),
                                                      ctypes.POINTER(ctypes.c_int64)]),
        "cl_batch_query": (ctypes.c_int, [vp]),
        "cl_observables": (ctypes.c_int, [vp, vp]),
        "cl_gauge_drift": (ctypes.c_int, [vp, dp, vp]),
        "cl_langevin_update": (ctypes.c_int, [vp, vp, vp, vp, vp, dp, dp, vp]),
        "cl_solve": (ctypes.c_int, [vp, vp, ctypes.c_int32, vp]),
        "cl_stochastic_blocks": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, vp]),
        "cl_drift_from_blocks": (ctypes.c_int, [vp, vp, vp]),
        "cl_batch_perturbations": (ctypes.c_int, [vp, i32p]),
        "cl_run_noalloc": (ctypes.c_int, [vp, ctypes.c_int32, vp, dp, dp, vp, vp, i32p, vp]),
        "cl_batch_inject_fault": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32]),
        "cl_batch_set_lanes": (ctypes.c_int, [vp, ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != CL_OK:
        L = lib()
        raise ClselError(rc, f"{L.cl_strerror(rc).decode()}: {L.cl_last_error().decode()}")


def _dims(dims):
    return (ctypes.c_int32 * 4)(*[int(v) for v in dims])


class Plan:
    """Symbolic analysis of one lattice shape (cl_symbolic_ex)."""

    def __init__(self, dims, leaf_sites: int = 0, max_pivot_rows: int = 0, nb: int = 0,
                 time_cuts: bool = False, gemm_tile: int = 0, lowrank_cap: int = 0,
                 pivot_floor: float = 0.0, smw_refine: int = 0):
        """pivot_floor: 0 takes the library default (0.3), a negative value turns pivot
        perturbation (and its low-rank correction) off; lowrank_cap: 0 takes the default;
        smw_refine: 1 refines the correction's solves once against D~ (default 0)."""
        L = lib()
        self.dims = tuple(int(v) for v in dims)
        self._h = ctypes.c_void_p()
        opts = PlanOpts(leaf_sites, max_pivot_rows, nb, 1 if time_cuts else 0, gemm_tile,
                        lowrank_cap, float(pivot_floor), int(smw_refine))
        _check(L.cl_symbolic_ex(_dims(dims), ctypes.byref(opts), ctypes.byref(self._h)))

    def info(self) -> dict:
        i = PlanInfo()
        _check(lib().cl_plan_info(self._h, ctypes.byref(i)))
        d = {k: getattr(i, k) for k, _ in PlanInfo._fields_}
        d["dims"] = tuple(i.dims)
        return d

    def bytes(self, batch: int) -> int:
        return int(lib().cl_plan_bytes(self._h, int(batch)))

    def export(self, what: int) -> np.ndarray:
        n = ctypes.c_size_t(0)
        _check(lib().cl_plan_export(self._h, what, None, ctypes.byref(n)))
        dt = {0: np.int64, 1: np.int32, 2: np.int32, 3: np.int32, 4: np.int64, 5: np.int64}[what]
        out = np.empty(n.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().cl_plan_export(self._h, what, out.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(n)))
        if what == 0:
            out = out.reshape(-1, len(FRONT_FIELDS))
        return out

    def fronts(self) -> list[dict]:
        return [dict(zip(FRONT_FIELDS, (int(v) for v in row))) for row in self.export(0)]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cl_plan_destroy(self._h)
            self._h = None


def run_noalloc(plan: "Plan", links, m, mu, selected_out=None, drift_out=None, stream=None):
    """cl_run_noalloc: the whole path for links [B][V][4][3][3] (complex128 GPU tensor) with
    every workspace in the library's static device array; no device memory is allocated by
    the library. Outputs are the caller's tensors (allocated here when not given, by torch).
    Returns (selected, drift, status) after the work has finished."""
    import torch
    B, V = int(links.shape[0]), int(plan.info()["volume"])
    if tuple(links.shape[1:]) != (V, 4, 3, 3):
        raise ClselError(CL_EINVAL, f"links must be [B][{V}][4][3][3]")
    if selected_out is None:
        selected_out = torch.empty((B, V, 9, 3, 3), dtype=torch.complex128, device=links.device)
    if drift_out is None:
        drift_out = torch.empty((B, V, 4, 8), dtype=torch.complex128, device=links.device)
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(m, dtype=np.float64), (B,)))
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,)))
    status = np.zeros(B, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().cl_run_noalloc(plan._h, B, _dev_ptr(links), m.ctypes.data_as(dp), mu.ctypes.data_as(dp),
                                _dev_ptr(selected_out), _dev_ptr(drift_out),
                                status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                _stream_handle(stream)))
    return selected_out, drift_out, status


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _dev_ptr(t, dtype_name="complex128"):
    import torch
    if not t.is_cuda or not t.is_contiguous() or t.dtype != getattr(torch, dtype_name):
        raise ClselError(CL_EINVAL, f"expected a contiguous {dtype_name} GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


class Batch:
    """Numeric workspace for `batch` configurations of one plan."""

    def __init__(self, plan: Plan, batch: int, stream=None):
        import torch
        self.plan = plan
        self.capacity = int(batch)
        self.active = int(batch)
        info = plan.info()
        self.V = int(info["volume"])
        self._h = ctypes.c_void_p()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().cl_batch_create(plan._h, self.capacity, _stream_handle(self._stream),
                                     ctypes.byref(self._h)))

    def set_active(self, n: int):
        _check(lib().cl_batch_set_active(self._h, int(n)))
        self.active = int(n)

    def set_lanes(self, lanes: int):
        """0: automatic; 1: one stream; 2: the second half of the configurations on a second
        stream of the batch (see cl_batch_set_lanes)."""
        _check(lib().cl_batch_set_lanes(self._h, int(lanes)))

    def use_graph(self, enable: bool = True):
        _check(lib().cl_batch_use_graph(self._h, 1 if enable else 0))

    def _params(self, m, mu):
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(m, dtype=np.float64), (self.active,)))
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (self.active,)))
        dp = ctypes.POINTER(ctypes.c_double)
        return m, mu, m.ctypes.data_as(dp), mu.ctypes.data_as(dp)

    def _check_links(self, links):
        if tuple(links.shape[-4:]) != (self.V, 4, 3, 3) or links.numel() < self.active * self.V * 36:
            raise ClselError(CL_EINVAL, f"links must be [B][{self.V}][4][3][3]")

    def factor(self, links, m, mu):
        self._check_links(links)
        _m, _mu, pm, pmu = self._params(m, mu)
        _check(lib().cl_factor(self._h, _dev_ptr(links), pm, pmu))

    def selinv(self):
        _check(lib().cl_selinv(self._h))

    def _alloc(self, shape):
        import torch
        return torch.empty(shape, dtype=torch.complex128, device="cuda")

    def selected(self, out=None):
        out = self._alloc((self.active, self.V, 9, 3, 3)) if out is None else out
        _check(lib().cl_selected(self._h, _dev_ptr(out)))
        return out

    def drift(self, out=None):
        out = self._alloc((self.active, self.V, 4, 8)) if out is None else out
        _check(lib().cl_drift(self._h, _dev_ptr(out)))
        return out

    def observables(self, out=None):
        """[B][2] complex128: (1/V) tr D^{-1} and (1/V) tr(D^{-1} dD/dmu)."""
        out = self._alloc((self.active, 2)) if out is None else out
        _check(lib().cl_observables(self._h, _dev_ptr(out)))
        return out

    def _per_config(self, v):
        v = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (self.active,)))
        return v, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def gauge_drift(self, beta, out=None):
        """[B][V][4][8] complex128: the Wilson gauge drift K^g of the links of the last
        factorisation (beta per configuration or scalar)."""
        out = self._alloc((self.active, self.V, 4, 8)) if out is None else out
        _b, pb = self._per_config(beta)
        _check(lib().cl_gauge_drift(self._h, pb, _dev_ptr(out)))
        return out

    def langevin_update(self, links_out, kf, eta, eps_bar, kref=None, kg=None, eps_out=None):
        """One Euler step of the links of the last factorisation into links_out:
        U <- exp[i sum_a lambda_a (eps K_a + sqrt(eps) eta_a)] U, K = kf (+ kg). eta is a
        real float64 [B][V][4][8] tensor; kref (per configuration, > 0) makes the step
        adaptive. Returns the [B] float64 tensor of steps used."""
        import torch
        self._check_links(links_out)
        if eps_out is None:
            eps_out = torch.empty((self.active,), dtype=torch.float64, device="cuda")
        _e, pe = self._per_config(eps_bar)
        if kref is not None:
            _k, pk = self._per_config(kref)
        else:
            pk = None
        _check(lib().cl_langevin_update(self._h, _dev_ptr(links_out), _dev_ptr(kf),
                                        _dev_ptr(kg) if kg is not None else None,
                                        _dev_ptr(eta, "float64"), pe, pk,
                                        _dev_ptr(eps_out, "float64")))
        return eps_out

    def solve(self, rhs, out=None):
        """X = D^{-1} rhs for rhs [B][N][n] complex128 (N = 3V) with the factors of the
        last factorisation."""
        if rhs.dim() != 3 or rhs.shape[0] < self.active or rhs.shape[1] != 3 * self.V:
            raise ClselError(CL_EINVAL, f"rhs must be [B][{3 * self.V}][n]")
        out = self._alloc((self.active, 3 * self.V, rhs.shape[2])) if out is None else out
        _check(lib().cl_solve(self._h, _dev_ptr(rhs), int(rhs.shape[2]), _dev_ptr(out)))
        return out

    def stochastic_blocks(self, xi, x, out=None):
        """Z~ = (1/n) X xi^dagger on the selected pattern, [B][V][9][3][3]."""
        out = self._alloc((self.active, self.V, 9, 3, 3)) if out is None else out
        _check(lib().cl_stochastic_blocks(self._h, _dev_ptr(xi), _dev_ptr(x), int(xi.shape[2]),
                                          _dev_ptr(out)))
        return out

    def drift_from_blocks(self, blocks, out=None):
        out = self._alloc((self.active, self.V, 4, 8)) if out is None else out
        _check(lib().cl_drift_from_blocks(self._h, _dev_ptr(blocks), _dev_ptr(out)))
        return out

    def run(self, links, m, mu, selected_out=None, drift_out=None, want_selected=True):
        self._check_links(links)
        if want_selected and selected_out is None:
            selected_out = self._alloc((self.active, self.V, 9, 3, 3))
        if drift_out is None:
            drift_out = self._alloc((self.active, self.V, 4, 8))
        _m, _mu, pm, pmu = self._params(m, mu)
        _check(lib().cl_run(self._h, _dev_ptr(links), pm, pmu,
                            _dev_ptr(selected_out) if selected_out is not None else None,
                            _dev_ptr(drift_out)))
        return selected_out, drift_out

    def profile(self, gemm_modes: int = 7):
        """Time GEMM launches of the modes in the bit mask (0 = off, 7 = every mode)."""
        _check(lib().cl_batch_profile(self._h, int(gemm_modes)))

    def profile_read(self):
        """(summed GEMM kernel ms, algorithmic flops, algorithmic bytes, launches) of the
        timed launches since the last read."""
        ms, fl, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().cl_batch_profile_read(self._h, ctypes.byref(ms), ctypes.byref(fl),
                                           ctypes.byref(by), ctypes.byref(n)))
        return ms.value, fl.value, by.value, n.value

    def profile_launches(self):
        """Per timed launch since the last profile_read: dict of arrays ms, flops, bytes, mode."""
        n = ctypes.c_int64()
        _check(lib().cl_batch_profile_launches(self._h, 0, None, None, None, None, ctypes.byref(n)))
        k = n.value
        ms, fl, by = (np.zeros(k) for _ in range(3))
        mode = np.zeros(k, dtype=np.int32)
        dptr = ctypes.POINTER(ctypes.c_double)
        _check(lib().cl_batch_profile_launches(
            self._h, k, ms.ctypes.data_as(dptr), fl.ctypes.data_as(dptr), by.ctypes.data_as(dptr),
            mode.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(n)))
        return {"ms": ms, "flops": fl, "bytes": by, "mode": mode}

    def status(self) -> np.ndarray:
        out = np.zeros(self.active, dtype=np.int32)
        _check(lib().cl_status(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def inject_fault(self, config: int, front: int):
        """Test support: zero the assembled pivot block of one front of one configuration in
        the following factorisations (front < 0: off)."""
        _check(lib().cl_batch_inject_fault(self._h, int(config), int(front)))

    def perturbations(self) -> np.ndarray:
        """Perturbed pivots of each active configuration in the last factorisation."""
        out = np.zeros(self.active, dtype=np.int32)
        _check(lib().cl_batch_perturbations(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def sync(self):
        _check(lib().cl_batch_sync(self._h))

    def done(self) -> bool:
        """True when the work of the last call has finished (does not block)."""
        rc = lib().cl_batch_query(self._h)
        if rc < 0:
            _check(rc)
        return rc == 1

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
