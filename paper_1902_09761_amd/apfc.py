"""Python binding of libapfc.so (include/apfc.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory (the workspace and
the amplitude tensors) and the stream.  There is no fallback: if the library is not built or
cannot be loaded, the functions raise.

Amplitude tensors are float64 CUDA tensors of shape (J, 2, N) (amplitude, re/im, node), nodes
in x-fastest order on the periodic uniform mesh.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int64, c_size_t, c_void_p
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapfc.so")

APFC_OK = 0
APFC_ERR_NOT_CONVERGED = 1
APFC_ERR_INVALID = -1
APFC_ERR_HIP = -2
APFC_ERR_WORKSPACE = -3
APFC_ERR_NONFINITE = -4
APFC_TRI2D, APFC_BCC3D, APFC_CUSTOM, APFC_FCC3D = 0, 1, 2, 3
APFC_FP64, APFC_MIXED = 0, 1
APFC_INNER_PCG, APFC_INNER_CHEB, APFC_INNER_MG = 0, 1, 2
APFC_MASS_ITER, APFC_MASS_SEPARABLE = 0, 1
APFC_OP_A, APFC_OP_PINV = 0, 1

EXPORTS = ["apfc_params_default", "apfc_lattice_default", "apfc_uniform_amplitude", "apfc_equilibrium_amplitudes",
           "apfc_create",
           "apfc_create_batch", "apfc_workspace_bytes", "apfc_set_workspace", "apfc_init_zeta", "apfc_step",
           "apfc_reset_history", "apfc_run",
           "apfc_energy", "apfc_energy_grad", "apfc_step_adjoint", "apfc_apply", "apfc_rotation", "apfc_probe_enable", "apfc_probe_read", "apfc_probe_read_kernel",
           "apfc_autotune", "apfc_set_tiles", "apfc_get_tiles", "apfc_set_graphs", "apfc_destroy", "apfc_status_string", "apfc_last_error",
           "apfc_step_noalloc", "apfc_noalloc_max_bytes"]


class apfc_mesh(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int64 * 3), ("length", c_double * 3)]


class apfc_lattice(ctypes.Structure):
    _fields_ = [("kind", c_int), ("J", c_int), ("k", (c_double * 3) * 8)]


class apfc_params(ctypes.Structure):
    _fields_ = [("a0", c_double), ("a1", c_double), ("a2", c_double), ("a3", c_double),
                ("picard_iters", c_int), ("rtol", c_double), ("restart", c_int), ("max_iters", c_int),
                ("precision", c_int), ("mass_iters", c_int), ("diff_iters", c_int), ("inner_kind", c_int),
                ("x0_order", c_int), ("mass_kind", c_int)]


class apfc_state(ctypes.Structure):
    _fields_ = [("eta", c_void_p), ("zeta", c_void_p)]


class apfc_stats(ctypes.Structure):
    _fields_ = [("total_iters", c_int), ("max_iters", c_int), ("cycles", c_int), ("max_relres", c_double),
                ("ms", c_double), ("iters", POINTER(c_int))]


class apfc_refine_params(ctypes.Structure):
    _fields_ = [("n_per_wavelength", c_double), ("grad_A_eps", c_double), ("A_min", c_double), ("h_int", c_double),
                ("h_max", c_double), ("tiny", c_double)]


class APFCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"apfc status {status}: {message}")
        self.status = status


class APFCNotConverged(APFCError):
    pass


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libapfc.so (built by paper_1902_09761_amd.build); raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1902_09761_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = POINTER
    sig = {
        "apfc_params_default": (None, [P(apfc_params)]),
        "apfc_lattice_default": (c_int, [c_int, P(apfc_lattice)]),
        "apfc_uniform_amplitude": (c_int, [P(apfc_lattice), P(apfc_params), P(c_double)]),
        "apfc_equilibrium_amplitudes": (c_int, [P(apfc_lattice), P(apfc_params), P(c_double)]),
        "apfc_create": (c_int, [P(apfc_mesh), P(apfc_lattice), P(apfc_params), P(c_void_p)]),
        "apfc_create_batch": (c_int, [c_int, P(apfc_mesh), P(apfc_lattice), P(apfc_params), P(c_void_p)]),
        "apfc_workspace_bytes": (c_size_t, [c_void_p]),
        "apfc_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
        "apfc_init_zeta": (c_int, [c_void_p, P(apfc_state), c_void_p]),
        "apfc_step": (c_int, [c_void_p, P(apfc_state), c_double, P(c_void_p), c_void_p, P(apfc_stats)]),
        "apfc_step_noalloc": (c_int, [c_void_p, P(apfc_state), c_double, P(c_void_p), c_void_p, P(apfc_stats)]),
        "apfc_noalloc_max_bytes": (c_size_t, []),
        "apfc_reset_history": (c_int, [c_void_p]),
        "apfc_run": (c_int, [c_void_p, P(apfc_state), c_double, c_int, P(c_void_p), c_void_p, P(apfc_stats),
                             P(c_int)]),
        "apfc_energy": (c_int, [c_void_p, P(apfc_state), P(c_double), c_void_p]),
        "apfc_energy_grad": (c_int, [c_void_p, P(apfc_state), P(c_void_p), P(c_double), c_void_p]),
        "apfc_step_adjoint": (c_int, [c_void_p, P(apfc_state), P(apfc_state), c_double, P(c_void_p),
                                      P(c_void_p), P(c_double), c_void_p, P(apfc_stats)]),
        "apfc_apply": (c_int, [c_void_p, c_int, P(apfc_state), P(apfc_state), P(apfc_state), c_double, c_void_p]),
        "apfc_rotation": (c_int, [c_void_p, P(apfc_state), P(c_void_p), P(c_void_p), P(apfc_refine_params), c_void_p]),
        "apfc_probe_enable": (c_int, [c_void_p, c_char_p, c_int]),
        "apfc_probe_read": (c_int, [c_void_p, P(c_int), P(c_double), P(c_double)]),
        "apfc_probe_read_kernel": (c_int, [c_void_p, c_char_p, P(c_int), P(c_double), P(c_double), P(c_int64)]),
        "apfc_autotune": (c_int, [c_void_p, c_void_p, P(c_int)]),
        "apfc_set_tiles": (c_int, [c_void_p, c_int, c_int]),
        "apfc_get_tiles": (c_int, [c_void_p, P(c_int), P(c_int)]),
        "apfc_set_graphs": (c_int, [c_void_p, c_int]),
        "apfc_destroy": (c_int, [c_void_p]),
        "apfc_status_string": (c_char_p, [c_int]),
        "apfc_last_error": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(rc: int):
    if rc == APFC_OK:
        return
    msg = lib().apfc_last_error().decode()
    if rc == APFC_ERR_NOT_CONVERGED:
        raise APFCNotConverged(rc, msg)
    raise APFCError(rc, msg)


# ---------------------------------------------------------------------------------------------
# same-name wrappers of the host-only calls
# ---------------------------------------------------------------------------------------------

def apfc_params_default(**overrides) -> apfc_params:
    p = apfc_params()
    lib().apfc_params_default(byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def apfc_lattice_default(kind: int) -> apfc_lattice:
    L = apfc_lattice()
    _check(lib().apfc_lattice_default(kind, byref(L)))
    return L


def lattice_k(L: apfc_lattice, dim: int):
    return [[L.k[j][d] for d in range(dim)] for j in range(L.J)]


def apfc_uniform_amplitude(lattice: apfc_lattice, params: apfc_params) -> float:
    phi = c_double()
    _check(lib().apfc_uniform_amplitude(byref(lattice), byref(params), byref(phi)))
    return phi.value


def apfc_noalloc_max_bytes() -> int:
    return int(lib().apfc_noalloc_max_bytes())


def apfc_equilibrium_amplitudes(lattice: apfc_lattice, params: apfc_params) -> List[float]:
    phi = (c_double * lattice.J)()
    _check(lib().apfc_equilibrium_amplitudes(byref(lattice), byref(params), phi))
    return list(phi)


def make_mesh(dim: int, n: Sequence[int], length: Sequence[float]) -> apfc_mesh:
    m = apfc_mesh()
    m.dim = dim
    for d in range(3):
        m.n[d] = int(n[d]) if d < len(n) else 1
        m.length[d] = float(length[d]) if d < len(length) else 1.0
    return m


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _ptr(t) -> c_void_p:
    return c_void_p(t.data_ptr())


def _check_field(t, J: int, N: int, name: str):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (J, 2, N)):
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of shape ({J}, 2, {N}), got "
                         f"{tuple(t.shape)} {t.dtype} {t.device}")


class Solver:
    """A batch of instances behind one apfc context (apfc_create_batch); one instance is a batch
    of one.  `meshes` and `params` are lists (params may be a single apfc_params)."""

    def __init__(self, meshes: List[apfc_mesh], lattice: apfc_lattice, params, device: str = "cuda",
                 attach_workspace: bool = True):
        """attach_workspace=False: no workspace tensor is allocated; only step_noalloc can run."""
        import torch
        if isinstance(meshes, apfc_mesh):
            meshes = [meshes]
        count = len(meshes)
        if isinstance(params, apfc_params):
            params = [params] * count
        self.count = count
        self.J = lattice.J
        self.dim = meshes[0].dim
        self.N = [int(m.n[0] * m.n[1] * (m.n[2] if m.dim == 3 else 1)) for m in meshes]
        marr = (apfc_mesh * count)(*meshes)
        parr = (apfc_params * count)(*params)
        self._lattice = lattice
        ctx = c_void_p()
        _check(lib().apfc_create_batch(count, marr, byref(lattice), parr, byref(ctx)))
        self.ctx = ctx
        nbytes = lib().apfc_workspace_bytes(ctx)
        self.workspace_bytes = nbytes
        self.workspace = None
        if attach_workspace:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            _check(lib().apfc_set_workspace(ctx, c_void_p(aligned), c_size_t(nbytes)))

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None and _LIB is not None:
                _LIB.apfc_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------------------
    def _states(self, etas, zetas=None):
        etas = list(etas)
        if len(etas) != self.count:
            raise ValueError(f"expected {self.count} instances")
        arr = (apfc_state * self.count)()
        for b, e in enumerate(etas):
            _check_field(e, self.J, self.N[b], "eta")
            arr[b].eta = e.data_ptr()
            if zetas is not None:
                _check_field(zetas[b], self.J, self.N[b], "zeta")
                arr[b].zeta = zetas[b].data_ptr()
        return arr

    def _ptrs(self, tensors, name):
        arr = (c_void_p * self.count)()
        for b, t in enumerate(tensors):
            _check_field(t, self.J, self.N[b], name)
            arr[b] = t.data_ptr()
        return arr

    # -- entry points --------------------------------------------------------------------
    def init_zeta(self, etas, zetas, stream=None):
        _check(lib().apfc_init_zeta(self.ctx, self._states(etas, zetas), _stream_handle(stream)))

    def reset_history(self):
        """Start a new trajectory for the extrapolated initial guess (params.x0_order > 0)."""
        _check(lib().apfc_reset_history(self.ctx))

    def step(self, etas, zetas, dt: float, source=None, stream=None) -> dict:
        st = apfc_stats()
        iters = (c_int * (self.count * self.J))()
        st.iters = ctypes.cast(iters, POINTER(c_int))
        src = self._ptrs(source, "source") if source is not None else None
        rc = lib().apfc_step(self.ctx, self._states(etas, zetas), float(dt), src, _stream_handle(stream), byref(st))
        info = {"total_iters": st.total_iters, "max_iters": st.max_iters, "cycles": st.cycles,
                "max_relres": st.max_relres, "ms": st.ms, "iters": list(iters)}
        if rc != APFC_OK:
            try:
                _check(rc)
            except APFCError as e:
                e.info = info
                raise
        return info

    def step_noalloc(self, etas, zetas, dt: float, source=None, stream=None) -> dict:
        """step() through apfc_step_noalloc (the library's static scratch instead of the workspace)."""
        st = apfc_stats()
        iters = (c_int * (self.count * self.J))()
        st.iters = ctypes.cast(iters, POINTER(c_int))
        src = self._ptrs(source, "source") if source is not None else None
        rc = lib().apfc_step_noalloc(self.ctx, self._states(etas, zetas), float(dt), src, _stream_handle(stream),
                                     byref(st))
        info = {"total_iters": st.total_iters, "max_iters": st.max_iters, "cycles": st.cycles,
                "max_relres": st.max_relres, "ms": st.ms, "iters": list(iters)}
        if rc != APFC_OK:
            try:
                _check(rc)
            except APFCError as e:
                e.info = info
                raise
        return info

    def run(self, etas, zetas, dt: float, nsteps: int, source=None, stream=None) -> dict:
        """nsteps steps in one call (apfc_run); info as step() plus step_max_iters per step."""
        st = apfc_stats()
        iters = (c_int * (self.count * self.J))()
        st.iters = ctypes.cast(iters, POINTER(c_int))
        per_step = (c_int * nsteps)()
        src = self._ptrs(source, "source") if source is not None else None
        rc = lib().apfc_run(self.ctx, self._states(etas, zetas), float(dt), int(nsteps), src,
                            _stream_handle(stream), byref(st), per_step)
        info = {"total_iters": st.total_iters, "max_iters": st.max_iters, "cycles": st.cycles,
                "max_relres": st.max_relres, "ms": st.ms, "iters": list(iters), "step_max_iters": list(per_step)}
        if rc != APFC_OK:
            try:
                _check(rc)
            except APFCError as e:
                e.info = info
                raise
        return info

    def energy(self, etas, stream=None) -> List[float]:
        out = (c_double * self.count)()
        _check(lib().apfc_energy(self.ctx, self._states(etas), out, _stream_handle(stream)))
        return list(out)

    def energy_grad(self, etas, grads, stream=None) -> List[float]:
        ddb = (c_double * self.count)()
        _check(lib().apfc_energy_grad(self.ctx, self._states(etas), self._ptrs(grads, "grad"), ddb,
                                      _stream_handle(stream)))
        return list(ddb)

    def step_adjoint(self, etas_before, etas_after, dt: float, lam_after, lam_before, stream=None) -> List[float]:
        ddb = (c_double * self.count)()
        st = apfc_stats()
        rc = lib().apfc_step_adjoint(self.ctx, self._states(etas_before), self._states(etas_after), float(dt),
                                     self._ptrs(lam_after, "lam_after"), self._ptrs(lam_before, "lam_before"), ddb,
                                     _stream_handle(stream), byref(st))
        _check(rc)
        return list(ddb)

    def apply(self, which: int, in_zetas, in_etas, out_zetas, out_etas, dt: float, lin_etas=None, stream=None):
        """out = A in (which = APFC_OP_A, linearised at lin_etas) or P^{-1} in (APFC_OP_PINV)."""
        lin = self._states(lin_etas) if lin_etas is not None else None
        _check(lib().apfc_apply(self.ctx, which, lin, self._states(in_etas, in_zetas),
                                self._states(out_etas, out_zetas), float(dt), _stream_handle(stream)))

    def rotation(self, etas, omegas, hs=None, n_per_wavelength=10.0, grad_A_eps=1e-2, A_min=1e-3, h_int=2.0,
                 h_max=40.0, tiny=1e-12, stream=None):
        """Local rotation omega (and the refinement indicator h) of every instance; omegas[b] is a
        float64 CUDA tensor of N (2D) or 3*N (3D) values, hs[b] of N values."""
        rp = apfc_refine_params(n_per_wavelength, grad_A_eps, A_min, h_int, h_max, tiny)
        om = (c_void_p * self.count)(*[o.data_ptr() for o in omegas])
        hp = (c_void_p * self.count)(*[t.data_ptr() for t in hs]) if hs is not None else None
        _check(lib().apfc_rotation(self.ctx, self._states(etas), om, hp, byref(rp), _stream_handle(stream)))

    def autotune(self, stream=None) -> int:
        ty = c_int()
        _check(lib().apfc_autotune(self.ctx, _stream_handle(stream), byref(ty)))
        return ty.value

    def set_tiles(self, tile_rows: int, precond_region: int = 0):
        _check(lib().apfc_set_tiles(self.ctx, int(tile_rows), int(precond_region)))

    def get_tiles(self):
        ty, reg = c_int(), c_int()
        _check(lib().apfc_get_tiles(self.ctx, byref(ty), byref(reg)))
        return ty.value, reg.value

    def set_graphs(self, enable: bool):
        _check(lib().apfc_set_graphs(self.ctx, 1 if enable else 0))

    def probe_enable(self, name: Optional[str], every: int = 1):
        _check(lib().apfc_probe_enable(self.ctx, name.encode() if name else None, every))

    def probe_read(self):
        n = c_int()
        ms = c_double()
        b = c_double()
        _check(lib().apfc_probe_read(self.ctx, byref(n), byref(ms), byref(b)))
        return n.value, ms.value, b.value

    def probe_read_kernel(self, name: str):
        """(sampled working launches, their total ms, mean algorithmic bytes, launches issued) of one
        kernel family since the last probe_read (which resets the records)."""
        n, ms, b, issued = c_int(), c_double(), c_double(), c_int64()
        _check(lib().apfc_probe_read_kernel(self.ctx, name.encode(), byref(n), byref(ms), byref(b), byref(issued)))
        return n.value, ms.value, b.value, issued.value
