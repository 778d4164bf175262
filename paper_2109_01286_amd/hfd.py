"""Python binding of ``libhfd.so`` (C ABI in ``include/hfd.h``).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Device memory and streams come from PyTorch (``torch.cuda``
tensors, ``torch.cuda.current_stream()``).  The library must be built
(``python -m paper_2109_01286_amd._build``); if it is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfd.so")

HFD_FP64, HFD_FP32_MIXED = 0, 1
SWITCH = {"paper": 0, "smooth": 1, "weno": 2}
FLUX = {"rusanov": 0, "roe": 1, "hllc": 2}
ORDER = {"none": 0, "hilbert": 1, "rcm": 2}
STATUS = {0: "HFD_OK", 1: "HFD_E_INVAL", 2: "HFD_E_MESH", 3: "HFD_E_NOMEM",
          4: "HFD_E_DEVICE", 5: "HFD_E_NUMERIC", 6: "HFD_E_STATE"}


class HfdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("gas_R", ctypes.c_double),
                ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("sw_lo", ctypes.c_double),
                ("sw_hi", ctypes.c_double), ("w3_cap", ctypes.c_double),
                ("period", ctypes.c_double * 2), ("w_ref", ctypes.c_double * 4),
                ("switch_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("order", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("stage_off", ctypes.c_int32), ("edge_grad", ctypes.c_int32),
                ("deg_inv", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class Info(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("n_owned", ctypes.c_int64),
                ("n_dirichlet", ctypes.c_int64), ("n_copy_ghost", ctypes.c_int64),
                ("n_edges_mesh", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_vslots", ctypes.c_int64), ("n_eslots", ctypes.c_int64),
                ("max_vslots", ctypes.c_int32), ("max_eslots", ctypes.c_int32),
                ("rank_hist", ctypes.c_int64 * 16), ("w3_truncated", ctypes.c_int64),
                ("bytes_edge_launch", ctypes.c_double),
                ("bytes_vertex_launch", ctypes.c_double),
                ("bytes_edge_w3_side", ctypes.c_double),
                ("setup_ms", ctypes.c_double * 4),
                ("stage_idx_bytes", ctypes.c_int32), ("stage_max_rows", ctypes.c_int32),
                ("stage_max_edges", ctypes.c_int32), ("reserved_info", ctypes.c_int32),
                ("bytes_vertex_staged", ctypes.c_double)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "hfd_default_opts": (None, [ctypes.POINTER(Opts)]),
    "hfd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hfd_last_error": (ctypes.c_char_p, [_P]),
    "hfd_create": (ctypes.c_int, [_P, _I64, _P, _I64, _P, ctypes.POINTER(Opts),
                                  ctypes.c_int, ctypes.POINTER(_P)]),
    "hfd_destroy": (ctypes.c_int, [_P]),
    "hfd_get_info": (ctypes.c_int, [_P, ctypes.POINTER(Info)]),
    "hfd_permutation": (ctypes.c_int, [_P, _P]),
    "hfd_export_edges": (ctypes.c_int, [_P, _P, _P]),
    "hfd_export_vertex_stencils": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "hfd_export_weights": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "hfd_import_weights": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "hfd_set_precision": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "hfd_set_flux": (ctypes.c_int, [_P, ctypes.c_int32]),
    "hfd_residual": (ctypes.c_int, [_P, _P, _P, _P]),
    "hfd_rk_step": (ctypes.c_int, [_P, _P, _D, _P]),
    "hfd_rk_step_dev": (ctypes.c_int, [_P, _P, _P, _P]),
    "hfd_rk_steps": (ctypes.c_int, [_P, _P, _I64, _D, _P, _P]),
    "hfd_stable_dt": (ctypes.c_int, [_P, _P, _D, _P, _P]),
    "hfd_stable_dt_noalloc": (ctypes.c_int, [_P, _P, _D, _P, _P]),
    "hfd_edge_states": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "hfd_export_grad_weights": (ctypes.c_int, [_P, _P, _P]),
    "hfd_import_grad_weights": (ctypes.c_int, [_P, _P, _P]),
    "hfd_force_switch_mask": (ctypes.c_int, [_P, _P]),
    "hfd_fill_ghosts": (ctypes.c_int, [_P, _P, _P]),
    "hfd_check": (ctypes.c_int, [_P, _P]),
    "hfd_adjoint_residual": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "hfd_rk_step_adjoint": (ctypes.c_int, [_P, _P, _D, _P, _P, _P]),
    "hfd_rk_step_stages": (ctypes.c_int, [_P, _P, _D, _P, _P, _P]),
    "hfd_rk_step_adjoint_stages": (ctypes.c_int, [_P, _P, _P, _P, _D, _P, _P, _P]),
    "hfd_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "hfd_kernel_times": (ctypes.c_int, [_P, _P, _P, _P, _P]),
}

_lib = None


def lib():
    """Load ``libhfd.so`` (once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2109_01286_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    """Host pointer of a contiguous numpy array (or None)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    """Device pointer of a torch tensor already checked by Solver._dev (or
    None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw):
    o = Opts()
    lib().hfd_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "switch":
            o.switch_mode = SWITCH[v] if isinstance(v, str) else int(v)
        elif k == "order":
            o.order = ORDER[v] if isinstance(v, str) else int(v)
        elif k == "flux":
            o.flux = FLUX[v] if isinstance(v, str) else int(v)
        elif k == "precision":
            o.precision = {"fp64": 0, "fp32": 1}[v] if isinstance(v, str) else int(v)
        elif k in ("period", "w_ref"):
            arr = getattr(o, k)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(o, k, v)
    return o


class Solver:
    """One mesh on one GPU.

    ``xy`` [V, 2] float64, ``tri`` [T, 3], ``ghost_src`` [V] (-1 owned, -2
    Dirichlet ghost, >= 0 copy source) in the caller's vertex numbering.
    States passed to the methods are torch float64 device tensors [12, V] in
    the library's internal order; :meth:`to_internal` / :meth:`to_input`
    convert.  ``device=-1`` builds the host-only setup (no GPU needed).
    """

    def __init__(self, xy, tri, ghost_src=None, period=(0.0, 0.0), device=0,
                 **opts):
        L = lib()
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        gs = None if ghost_src is None else np.ascontiguousarray(ghost_src, np.int32)
        self.opts = default_opts(period=period, **opts)
        h = ctypes.c_void_p()
        st = L.hfd_create(_ptr(xy), xy.shape[0], _ptr(tri), tri.shape[0], _ptr(gs),
                          ctypes.byref(self.opts), int(device), ctypes.byref(h))
        if st != 0:
            raise HfdError(st, L.hfd_last_error(None).decode())
        self._h = h
        self.device = device
        inf = Info()
        self._chk(L.hfd_get_info(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()
        self.nv = self.info["nv"]
        self.n_owned = self.info["n_owned"]
        self.ne = self.info["n_edges"]
        perm = np.empty(self.nv, dtype=np.int32)
        self._chk(L.hfd_permutation(self._h, _ptr(perm)))
        self.new_of_old = perm.astype(np.int64)
        self.old_of_new = np.empty_like(self.new_of_old)
        self.old_of_new[self.new_of_old] = np.arange(self.nv)
        self._dt_buf = None
        self._force = None

    # -- plumbing -------------------------------------------------------------
    def _chk(self, st):
        if st != 0:
            raise HfdError(st, lib().hfd_last_error(self._h).decode())

    def _dev(self, t, name, dtype="float64", shape=None, min_numel=None):
        """Check one device argument before anything is launched: a torch
        tensor of the given dtype and shape (or at least ``min_numel``
        elements), contiguous, on this solver's GPU.  The C ABI takes bare
        pointers and cannot see any of this, so a wrong tensor would make
        the kernels read or write past its end.  Raises ValueError."""
        import torch
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        want = getattr(torch, dtype)
        if t.dtype != want:
            raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
        if min_numel is not None and t.numel() < min_numel:
            raise ValueError(f"{name}: {t.numel()} elements, at least {min_numel} expected")
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name}: on {t.device}, expected cuda:{self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: not contiguous")
        return _dptr(t)

    def _state(self, t, name="U"):
        return self._dev(t, name, shape=(12, self.nv))

    def close(self):
        if getattr(self, "_h", None):
            lib().hfd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh_info(self):
        inf = Info()
        self._chk(lib().hfd_get_info(self._h, ctypes.byref(inf)))
        self.info = inf.as_dict()
        return self.info

    # -- numbering ----------------------------------------------------------------
    def to_internal(self, U):
        """[12, V] in input order -> internal order (numpy or torch)."""
        if isinstance(U, np.ndarray):
            return np.ascontiguousarray(U[:, self.old_of_new])
        import torch
        idx = torch.as_tensor(self.old_of_new, device=U.device)
        return U[:, idx].contiguous()

    def to_input(self, U):
        if isinstance(U, np.ndarray):
            return np.ascontiguousarray(U[:, self.new_of_old])
        import torch
        idx = torch.as_tensor(self.new_of_old, device=U.device)
        return U[:, idx].contiguous()

    # -- setup exports --------------------------------------------------------------
    def export_edges(self):
        ends = np.empty((self.ne, 2), dtype=np.int32)
        st = np.empty((self.ne, 6), dtype=np.int32)
        self._chk(lib().hfd_export_edges(self._h, _ptr(ends), _ptr(st)))
        return ends, st

    def export_vertex_stencils(self):
        no = self.n_owned
        vptr = np.empty(no + 1, dtype=np.int64)
        eptr = np.empty(no + 1, dtype=np.int64)
        vn = np.empty(self.info["n_vslots"], dtype=np.int32)
        ve = np.empty(self.info["n_eslots"], dtype=np.int32)
        self._chk(lib().hfd_export_vertex_stencils(self._h, _ptr(vptr), _ptr(vn),
                                                   _ptr(eptr), _ptr(ve)))
        return vptr, vn, eptr, ve

    def export_weights(self):
        ne, nvs, nes = self.ne, self.info["n_vslots"], self.info["n_eslots"]
        w5 = np.empty((ne, 2, 15))
        w3 = np.empty((ne, 2, 3, 3))
        rank = np.empty((ne, 2), dtype=np.int32)
        dv = np.empty((nvs, 6))
        de = np.empty((nes, 3))
        dvis = np.empty((nvs, 5)) if self.opts.mu > 0 else None
        self._chk(lib().hfd_export_weights(self._h, _ptr(w5), _ptr(w3), _ptr(rank),
                                           _ptr(dv), _ptr(de), _ptr(dvis)))
        return dict(w5=w5, w3=w3, rank=rank, dv=dv, de=de, dvis=dvis)

    def import_weights(self, w5=None, w3=None, dv=None, de=None, dvis=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        w5, w3, dv, de, dvis = map(c, (w5, w3, dv, de, dvis))
        self._chk(lib().hfd_import_weights(self._h, _ptr(w5), _ptr(w3), _ptr(dv),
                                           _ptr(de), _ptr(dvis)))

    def export_grad_weights(self):
        ne = self.ne
        w5g = np.empty((ne, 2, 2, 15))
        w3g = np.empty((ne, 2, 3, 2, 3))
        self._chk(lib().hfd_export_grad_weights(self._h, _ptr(w5g), _ptr(w3g)))
        return dict(w5g=w5g, w3g=w3g)

    def import_grad_weights(self, w5g=None, w3g=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        w5g, w3g = c(w5g), c(w3g)
        for a, shp in ((w5g, (self.ne, 2, 2, 15)), (w3g, (self.ne, 2, 3, 2, 3))):
            if a is not None and a.shape != shp:
                raise ValueError(f"shape {a.shape}, expected {shp}")
        self._chk(lib().hfd_import_grad_weights(self._h, _ptr(w5g), _ptr(w3g)))

    def set_precision(self, precision, w_ref=None):
        p = {"fp64": 0, "fp32": 1}[precision] if isinstance(precision, str) else precision
        wr = None if w_ref is None else np.ascontiguousarray(w_ref, dtype=np.float64)
        self._chk(lib().hfd_set_precision(self._h, int(p), _ptr(wr)))
        self.opts.precision = int(p)
        self.refresh_info()

    def set_flux(self, flux):
        """Riemann flux of later calls: "rusanov", "roe" or "hllc"."""
        f = FLUX[flux] if isinstance(flux, str) else int(flux)
        self._chk(lib().hfd_set_flux(self._h, f))
        self.opts.flux = f

    # -- hot path -------------------------------------------------------------------
    # Every device argument is checked by _dev / _state before the call.
    def residual(self, U, out=None):
        import torch
        pU = self._state(U)
        if out is None:
            out = torch.empty_like(U)
        self._chk(lib().hfd_residual(self._h, pU, self._state(out, "out"), _stream()))
        return out

    def rk_step(self, U, dt):
        """One RK3 step in place; ``dt`` a float or a 1-element device tensor."""
        import torch
        pU = self._state(U)
        if isinstance(dt, torch.Tensor):
            pdt = self._dev(dt, "dt", min_numel=1)
            self._chk(lib().hfd_rk_step_dev(self._h, pU, pdt, _stream()))
        else:
            self._chk(lib().hfd_rk_step(self._h, pU, float(dt), _stream()))
        return U

    def rk_steps(self, U, nsteps, cfl, dts=None):
        """nsteps x (stable_dt then rk_step) in place; returns the device
        tensor [nsteps] of step sizes (no host sync)."""
        import torch
        nsteps = int(nsteps)
        if nsteps < 0:
            raise ValueError(f"nsteps = {nsteps} < 0")
        pU = self._state(U)
        if dts is None:
            dts = torch.empty(max(nsteps, 1), dtype=torch.float64, device=U.device)
        pd = self._dev(dts, "dts", min_numel=max(nsteps, 1))
        self._chk(lib().hfd_rk_steps(self._h, pU, nsteps, float(cfl), pd, _stream()))
        return dts

    def capture_steps(self, U, nsteps, cfl, dts):
        """A HIP graph (torch.cuda.CUDAGraph) of ``nsteps`` x (device-side
        time step, Runge-Kutta step) on U in place, the step sizes going to
        dts[:nsteps]: ``g.replay()`` runs them again on the same buffers,
        with one launch from the host.  The library's kernels are all that is
        captured (the call allocates, copies and clears nothing), so the
        pass timing must be off.  Nothing runs at capture."""
        import torch
        if getattr(self, "_timing", False):
            raise ValueError("capture_steps: pass timing is on (set_timing(False))")
        self._state(U)
        self._dev(dts, "dts", min_numel=max(int(nsteps), 1))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.rk_steps(U, nsteps, cfl, dts)
        return g

    def stable_dt(self, U, cfl, out=None):
        """Device tensor [1] with cfl * min h/(|u|+c) (no host sync)."""
        import torch
        pU = self._state(U)
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=U.device)
        self._chk(lib().hfd_stable_dt(self._h, pU, float(cfl),
                                      self._dev(out, "out", min_numel=1), _stream()))
        return out

    def stable_dt_noalloc(self, U, cfl, out):
        """stable_dt into the caller's device tensor ``out`` [>= 1] through
        the entry point that allocates nothing (library scratch; calls on
        one GPU must not overlap)."""
        self._chk(lib().hfd_stable_dt_noalloc(self._h, self._state(U), float(cfl),
                                              self._dev(out, "out", min_numel=1), _stream()))
        return out

    def edge_states(self, U, want_mask=True, want_flux=True, want_grad=False):
        """(wlr [8, ne], mask [ne] or None, h [4, ne] or None), and with
        ``want_grad`` also grad [16, ne] (needs ``edge_grad=1``)."""
        import torch
        pU = self._state(U)
        wlr = torch.empty(8, self.ne, dtype=torch.float64, device=U.device)
        mask = torch.empty(self.ne, dtype=torch.uint8, device=U.device) if want_mask else None
        h = torch.empty(4, self.ne, dtype=torch.float64, device=U.device) if want_flux else None
        g = torch.empty(16, self.ne, dtype=torch.float64, device=U.device) if want_grad else None
        self._chk(lib().hfd_edge_states(self._h, pU, _dptr(wlr), _dptr(g), _dptr(mask),
                                        _dptr(h), _stream()))
        return (wlr, mask, h, g) if want_grad else (wlr, mask, h)

    def force_switch_mask(self, mask):
        """Force the Hermite/WENO branch per edge (uint8 device tensor [ne])
        or return to the configured switch (None)."""
        p = None if mask is None else self._dev(mask, "mask", dtype="uint8", shape=(self.ne,))
        self._force = mask
        self._chk(lib().hfd_force_switch_mask(self._h, p))

    def adjoint_residual(self, U, lam, out=None):
        """(dR/dU)^T lam (float64 device tensors [12, V], internal order),
        computed in the context's precision."""
        import torch
        pU, pl = self._state(U), self._state(lam, "lam")
        if out is None:
            out = torch.empty_like(U)
        self._chk(lib().hfd_adjoint_residual(self._h, pU, pl, self._state(out, "out"),
                                             _stream()))
        return out

    def rk_step_adjoint(self, U_n, dt, lam_np1, out=None):
        """(dU_{n+1}/dU_n)^T lam_np1 for one RK3 step of size dt from U_n."""
        import torch
        pU, pl = self._state(U_n, "U_n"), self._state(lam_np1, "lam_np1")
        if out is None:
            out = torch.empty_like(U_n)
        self._chk(lib().hfd_rk_step_adjoint(self._h, pU, float(dt), pl,
                                            self._state(out, "out"), _stream()))
        return out

    def rk_step_stages(self, U, dt, U1, U2):
        """One RK3 step in place (the context's precision) that also writes
        its intermediate stages into U1, U2 (device tensors shaped like U)."""
        self._chk(lib().hfd_rk_step_stages(self._h, self._state(U), float(dt),
                                           self._state(U1, "U1"), self._state(U2, "U2"),
                                           _stream()))
        return U

    def rk_step_adjoint_stages(self, U_n, U1, U2, dt, lam_np1, out=None):
        """rk_step_adjoint with the step's stages (from rk_step_stages) given."""
        import torch
        p = [self._state(U_n, "U_n"), self._state(U1, "U1"), self._state(U2, "U2")]
        pl = self._state(lam_np1, "lam_np1")
        if out is None:
            out = torch.empty_like(U_n)
        self._chk(lib().hfd_rk_step_adjoint_stages(self._h, *p, float(dt), pl,
                                                   self._state(out, "out"), _stream()))
        return out

    def fill_ghosts(self, U):
        self._chk(lib().hfd_fill_ghosts(self._h, self._state(U), _stream()))
        return U

    def check(self):
        self._chk(lib().hfd_check(self._h, _stream()))

    def set_timing(self, on=True):
        self._chk(lib().hfd_set_timing(self._h, int(bool(on))))
        self._timing = bool(on)

    def kernel_times(self):
        """(edge_ms_total, n_edge, vertex_ms_total, n_vertex) since last call."""
        e, v = ctypes.c_double(), ctypes.c_double()
        ne_, nv_ = ctypes.c_int64(), ctypes.c_int64()
        self._chk(lib().hfd_kernel_times(self._h, ctypes.byref(e), ctypes.byref(ne_),
                                         ctypes.byref(v), ctypes.byref(nv_)))
        return e.value, ne_.value, v.value, nv_.value
