"""Thin Python binding of ``libpf.so`` (argument marshalling only).

Every function mirrors the C entry point of the same name in
``include/pf.h``; all computation happens in the library's HIP kernels.
Device arrays are ``torch`` float64 CUDA tensors (PyTorch provides device
memory and streams only); ``stream=None`` means torch's current stream.
The library must be built (``python -m paper_2302_10736_amd.build``):
without it the first call raises ImportError; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_ESTATE, PF_EUNSUP = range(6)
PF_METHOD_ELEMENTWISE, PF_METHOD_YBUS, PF_METHOD_ELEMENTWISE_TWO_PHASE, PF_METHOD_ELEMENTWISE_ATOMIC = 0, 1, 2, 3
PF_BUILD_HOST_ONLY = 1
PF_ORDER_AUTO, PF_ORDER_TILE_MAJOR, PF_ORDER_STATE_MAJOR, PF_ORDER_GROUPED = 0, 1, 2, 3
PF_PHASOR_SPLIT, PF_PHASOR_INTERLEAVED = 1, 2
PF_JAC_CSC = 0x100  # OR into the method of pf_jacobian_values: J values in CSC order
PF_LAYOUT_CSR, PF_LAYOUT_CSC = 0, 1
PF_EW_PRECOMPUTED = 0x200  # OR into the two-phase / copy-add methods: precomputed branch constants

EXPORTS = (
    "pf_build_pattern", "pf_grid_free", "pf_grid_sizes", "pf_pattern_sizes", "pf_grid_offsets",
    "pf_pattern_export", "pf_ybus", "pf_injections_elementwise", "pf_injections_ybus", "pf_jacobian_values",
    "pf_injections_vjp", "pf_jacobian_two_phase_static", "pf_branch_flows", "pf_phasors", "pf_ybus_from_phasors", "pf_jacobian_map", "pf_jacobian_scatter", "pf_set_schedule", "pf_get_schedule", "pf_graph_create", "pf_graph_launch",
    "pf_graph_free", "pf_autotune", "pf_stream_copy", "pf_debug_fail_allocs", "pf_last_error", "pf_version",
)
PF_OP_INJECTIONS, PF_OP_JACOBIAN, PF_OP_VJP = 0, 1, 2


class PfOp(C.Structure):
    """``pf_op`` of include/pf.h."""
    _fields_ = [("op", C.c_int32), ("method", C.c_int32), ("nstate", C.c_int32),
                ("vm", C.c_void_p), ("va", C.c_void_p), ("lam_p", C.c_void_p), ("lam_q", C.c_void_p),
                ("out_a", C.c_void_p), ("out_b", C.c_void_p), ("jval", C.c_void_p)]


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pf error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2302_10736_amd.build`")
        # torch bundles its own HIP runtime with the same soname; loading it
        # first makes libpf.so bind to it, so the process holds one runtime.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        L.pf_build_pattern.argtypes = [i32, i32] + [P] * 9 + [i32, P, P, u32, C.POINTER(P)]
        L.pf_grid_free.argtypes = [P]
        L.pf_grid_free.restype = None
        L.pf_grid_sizes.argtypes = [P, P, P, P, P]
        L.pf_pattern_sizes.argtypes = [P, P, P]
        L.pf_grid_offsets.argtypes = [P, P, P]
        L.pf_pattern_export.argtypes = [P, P, P, P, P]
        L.pf_ybus.argtypes = [P, P, P, P]
        L.pf_injections_elementwise.argtypes = [P, i32, P, P, P, P, P]
        L.pf_injections_ybus.argtypes = [P, i32, P, P, P, P, P]
        L.pf_jacobian_values.argtypes = [P, i32, i32, P, P, P, P, P, P]
        L.pf_injections_vjp.argtypes = [P, i32, P, P, P, P, P, P, P]
        L.pf_jacobian_two_phase_static.argtypes = [P, i32, i32, P, P, P, P, P, P]
        L.pf_branch_flows.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.pf_phasors.argtypes = [P, i32, i32, P, P, P, P]
        L.pf_jacobian_map.argtypes = [P, i32, i32, P, P, P]
        L.pf_jacobian_scatter.argtypes = [P, i32, P, P, i64, P, P]
        L.pf_stream_copy.argtypes = [P, P, i64, P]
        L.pf_debug_fail_allocs.argtypes = [i32]
        L.pf_ybus_from_phasors.argtypes = [P, i32, i32, P, P, P, P, P]
        L.pf_set_schedule.argtypes = [P, i32, i32, i32]
        L.pf_graph_create.argtypes = [P, P, i32, C.POINTER(P)]
        L.pf_graph_launch.argtypes = [P, P]
        L.pf_graph_free.argtypes = [P]
        L.pf_graph_free.restype = None
        L.pf_autotune.argtypes = [P, P, i32, P, i32, P, P, P]
        L.pf_get_schedule.argtypes = [P, P, P, P, P]
        L.pf_last_error.restype = C.c_char_p
        L.pf_last_error.argtypes = []
        L.pf_version.restype = C.c_char_p
        L.pf_version.argtypes = []
        for name in EXPORTS:
            if name not in ("pf_grid_free", "pf_graph_free", "pf_last_error", "pf_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != PF_OK:
        raise PFError(rc, lib().pf_last_error().decode())


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, shape=None, name="array"):
    """Device pointer of a float64 CUDA tensor (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


class Grid:
    """Owner of a ``pf_grid`` handle (pf_build_pattern / pf_grid_free)."""

    def __init__(self, nb, nl, fbus, tbus, r, x, b, tap, shift, gs=None, bs=None, bus_off=None, br_off=None,
                 host_only=False):
        self._h = C.c_void_p()
        arrs = [_host(fbus, np.int32), _host(tbus, np.int32)] + [_host(a, np.float64) for a in (r, x, b, tap, shift)]
        gsa, bsa = _host(gs, np.float64), _host(bs, np.float64)
        bo, ro = _host(bus_off, np.int32), _host(br_off, np.int32)
        ngrids = 1 if bo is None else len(bo) - 1
        self._keep = (arrs, gsa, bsa, bo, ro)
        check(lib().pf_build_pattern(int(nb), int(nl), *[_hp(a) for a in arrs], _hp(gsa), _hp(bsa), ngrids,
                                     _hp(bo), _hp(ro), PF_BUILD_HOST_ONLY if host_only else 0, C.byref(self._h)))
        self._keep = None
        n_b, n_y, n_j, n_g = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        check(lib().pf_grid_sizes(self._h, C.byref(n_b), C.byref(n_y), C.byref(n_j), C.byref(n_g)))
        self.nb, self.nnz_y, self.nnz_j, self.ngrids = n_b.value, n_y.value, n_j.value, n_g.value
        self.nl = int(nl)

    @classmethod
    def from_grid(cls, g, bus_off=None, br_off=None, host_only=False):
        """From any object with nb, nl, fbus, tbus, r, x, b, tap, shift, gs, bs."""
        return cls(g.nb, g.nl, g.fbus, g.tbus, g.r, g.x, g.b, g.tap, g.shift, g.gs, g.bs, bus_off, br_off,
                   host_only)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            lib().pf_grid_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def offsets(self):
        y = np.zeros(self.ngrids + 1, np.int64)
        j = np.zeros(self.ngrids + 1, np.int64)
        check(lib().pf_grid_offsets(self._h, _hp(y), _hp(j)))
        return y, j

    def pattern(self):
        """(y_rowptr, y_col, j_rowptr, j_col), grid after grid, grid-local indices."""
        yr = np.zeros(self.nb + self.ngrids, np.int32)
        yc = np.zeros(max(self.nnz_y, 1), np.int32)
        jr = np.zeros(2 * self.nb + self.ngrids, np.int32)
        jc = np.zeros(max(self.nnz_j, 1), np.int32)
        check(lib().pf_pattern_export(self._h, _hp(yr), _hp(yc), _hp(jr), _hp(jc)))
        return yr, yc[: self.nnz_y], jr, jc[: self.nnz_j]

    def set_schedule(self, tile_items=256, states_per_block=0, order=PF_ORDER_AUTO):
        check(lib().pf_set_schedule(self._h, int(tile_items), int(states_per_block), int(order)))

    def schedule(self):
        """(tile_items, states_per_block, order, ntiles)."""
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().pf_get_schedule(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, d.value


def _nstate(vm, nb):
    if vm.dim() == 1:
        if vm.shape[0] != nb:
            raise ValueError("state length differs from nb")
        return 1
    if vm.dim() != 2 or vm.shape[1] != nb:
        raise ValueError("states must be [nstate, nb]")
    return vm.shape[0]


def pf_build_pattern(nb, nl, fbus, tbus, r, x, b, tap, shift, gs=None, bs=None, bus_off=None, br_off=None,
                     host_only=False) -> Grid:
    return Grid(nb, nl, fbus, tbus, r, x, b, tap, shift, gs, bs, bus_off, br_off, host_only)


def pf_ybus(grid: Grid, y_re=None, y_im=None, stream=None):
    check(lib().pf_ybus(grid.handle, _dev(y_re, (grid.nnz_y,), "y_re"), _dev(y_im, (grid.nnz_y,), "y_im"),
                        _stream(stream)))


def _m_injections_elementwise(grid: Grid, vm, va, p, q, stream=None):
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    return (grid.handle, ns, _dev(vm, shp, "vm"), _dev(va, shp, "va"), _dev(p, shp, "p"), _dev(q, shp, "q"),
            _stream(stream))


def _m_injections_ybus(grid: Grid, vm, va, p, q, stream=None):
    return _m_injections_elementwise(grid, vm, va, p, q, stream)


def _m_jacobian_values(grid: Grid, method: int, vm, va, p, q, jval, stream=None):
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    jshp = (grid.nnz_j,) if vm.dim() == 1 else (ns, grid.nnz_j)
    return (grid.handle, int(method), ns, _dev(vm, shp, "vm"), _dev(va, shp, "va"), _dev(p, shp, "p"),
            _dev(q, shp, "q"), _dev(jval, jshp, "jval"), _stream(stream))


def _m_injections_vjp(grid: Grid, vm, va, lam_p, lam_q, g_vm, g_va, stream=None):
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    return (grid.handle, ns, _dev(vm, shp, "vm"), _dev(va, shp, "va"), _dev(lam_p, shp, "lam_p"),
            _dev(lam_q, shp, "lam_q"), _dev(g_vm, shp, "g_vm"), _dev(g_va, shp, "g_va"), _stream(stream))


def _m_branch_flows(grid: Grid, vm, va, pf_, qf, pt, qt, jac=None, stream=None):
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    nl = grid.nl
    fshp = (nl,) if vm.dim() == 1 else (ns, nl)
    jshp = (16, nl) if vm.dim() == 1 else (ns, 16, nl)
    return (grid.handle, ns, _dev(vm, shp, "vm"), _dev(va, shp, "va"), _dev(pf_, fshp, "pf"), _dev(qf, fshp, "qf"),
            _dev(pt, fshp, "pt"), _dev(qt, fshp, "qt"), _dev(jac, jshp, "jac"), _stream(stream))


def pf_injections_elementwise(grid: Grid, vm, va, p, q, stream=None):
    check(lib().pf_injections_elementwise(*_m_injections_elementwise(grid, vm, va, p, q, stream)))


def pf_injections_ybus(grid: Grid, vm, va, p, q, stream=None):
    check(lib().pf_injections_ybus(*_m_injections_ybus(grid, vm, va, p, q, stream)))


def pf_jacobian_values(grid: Grid, method: int, vm, va, p, q, jval, stream=None):
    check(lib().pf_jacobian_values(*_m_jacobian_values(grid, method, vm, va, p, q, jval, stream)))


def pf_jacobian_two_phase_static(grid: Grid, method: int, vm, va, p, q, jval, stream=None):
    """The two-phase Jacobian with the library's static scratch (allocates
    nothing; see include/pf.h for the size limit and the sharing rule)."""
    check(lib().pf_jacobian_two_phase_static(*_m_jacobian_values(grid, method, vm, va, p, q, jval, stream)))


def pf_injections_vjp(grid: Grid, vm, va, lam_p, lam_q, g_vm, g_va, stream=None):
    check(lib().pf_injections_vjp(*_m_injections_vjp(grid, vm, va, lam_p, lam_q, g_vm, g_va, stream)))


def pf_branch_flows(grid: Grid, vm, va, pf_, qf, pt, qt, jac=None, stream=None):
    check(lib().pf_branch_flows(*_m_branch_flows(grid, vm, va, pf_, qf, pt, qt, jac, stream)))


_MARSHAL = {
    "pf_injections_elementwise": _m_injections_elementwise,
    "pf_injections_ybus": _m_injections_ybus,
    "pf_jacobian_values": _m_jacobian_values,
    "pf_injections_vjp": _m_injections_vjp,
    "pf_branch_flows": _m_branch_flows,
}


class Bound:
    """One evaluation call with its arguments checked and marshalled once.

    Calling the object only calls the library function with the stored
    arguments: for loops that evaluate again and again on the same buffers
    (their contents may change between calls), where the per-call argument
    checks of the plain binding cost more host time than the kernel.  The
    stream is fixed when binding (``stream=None``: torch's current stream at
    that moment).  The object keeps the grid and the tensors alive."""

    def __init__(self, fn, *args, **kw):
        name = getattr(fn, "__name__", fn)
        if name not in _MARSHAL:
            raise ValueError(f"cannot bind {name!r}; one of {sorted(_MARSHAL)}")
        self._f = getattr(lib(), name)
        self._args = _MARSHAL[name](*args, **kw)
        self._keep = (args, kw)

    def __call__(self):
        rc = self._f(*self._args)
        if rc != PF_OK:
            raise PFError(rc, lib().pf_last_error().decode())


def bind(fn, *args, **kw) -> Bound:
    """``bind(pf_jacobian_values, grid, method, vm, va, p, q, jval)`` returns a
    :class:`Bound` call; the arguments are those of ``fn``."""
    return Bound(fn, *args, **kw)


def pf_phasors(grid: Grid, layout: int, vm, va, ph, stream=None):
    """V and U of every state into ``ph`` (float64, 4 * nstate * nb values,
    any shape): see include/pf.h for the two layouts."""
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    if ph.numel() != 4 * ns * grid.nb:
        raise ValueError("ph must hold 4 * nstate * nb values")
    check(lib().pf_phasors(grid.handle, int(layout), ns, _dev(vm, shp, "vm"), _dev(va, shp, "va"),
                           _dev(ph, None, "ph"), _stream(stream)))


def pf_ybus_from_phasors(grid: Grid, layout: int, nstate: int, ph, p=None, q=None, jval=None, stream=None):
    """Ybus injections (and Jacobian values if ``jval`` is given) from the
    phasors ``pf_phasors`` wrote; ``nstate`` states, outputs [nstate, nb] /
    [nstate, nnz_j] (or 1-D for one state)."""
    if ph.numel() != 4 * nstate * grid.nb:
        raise ValueError("ph must hold 4 * nstate * nb values")
    ref = p if p is not None else jval
    flat = ref is not None and ref.dim() == 1
    shp = (grid.nb,) if flat else (nstate, grid.nb)
    jshp = (grid.nnz_j,) if flat else (nstate, grid.nnz_j)
    check(lib().pf_ybus_from_phasors(grid.handle, int(layout), int(nstate), _dev(ph, None, "ph"), _dev(p, shp, "p"),
                                     _dev(q, shp, "q"), _dev(jval, jshp, "jval"), _stream(stream)))


def pf_jacobian_map(grid: Grid, layout: int, ptr, idx) -> np.ndarray:
    """Positions of J's entries (exported CSR order) in a target pattern of
    size 2 nb (host arrays; CSR row pointers and column indices, or CSC
    column pointers and row indices); returns int32[nnz_j]."""
    ptr = _host(ptr, np.int32)
    idx = _host(idx, np.int32)
    if ptr is None or idx is None or ptr.ndim != 1 or len(ptr) < 1:
        raise ValueError("ptr and idx must be 1-D arrays")
    out = np.empty(max(grid.nnz_j, 1), np.int32)
    check(lib().pf_jacobian_map(grid.handle, int(layout), len(ptr) - 1, _hp(ptr), _hp(idx if len(idx) else np.zeros(1, np.int32)),
                                _hp(out)))
    return out[: grid.nnz_j]


def pf_jacobian_scatter(grid: Grid, jval, jmap, out, stream=None):
    """out[s, jmap[k]] = jval[s, k] (device tensors: jval float64 [nstate,
    nnz_j] or [nnz_j], jmap int32 [nnz_j], out float64 [nstate, out_nnz] or
    [out_nnz])."""
    import torch
    if not isinstance(jmap, torch.Tensor) or jmap.dtype != torch.int32 or not jmap.is_cuda \
            or not jmap.is_contiguous() or tuple(jmap.shape) != (grid.nnz_j,):
        raise ValueError("jmap must be a contiguous int32 CUDA tensor of nnz_j entries")
    ns = 1 if jval.dim() == 1 else jval.shape[0]
    jshp = (grid.nnz_j,) if jval.dim() == 1 else (ns, grid.nnz_j)
    out_nnz = out.shape[-1]
    oshp = (out_nnz,) if jval.dim() == 1 else (ns, out_nnz)
    check(lib().pf_jacobian_scatter(grid.handle, ns, _dev(jval, jshp, "jval"), C.c_void_p(jmap.data_ptr()),
                                    int(out_nnz), _dev(out, oshp, "out"), _stream(stream)))


def pf_stream_copy(src, dst, stream=None):
    """dst[:] = src[:] by the library's streaming copy kernel (measurement
    aid: the bandwidth ceiling at a byte count).  Contiguous float64 CUDA
    tensors of equal size, 16-byte aligned, not overlapping."""
    if src is None or dst is None or src.numel() != dst.numel():
        raise ValueError("src and dst must be tensors of equal size")
    n = src.numel()
    check(lib().pf_stream_copy(_dev(src, tuple(src.shape), "src"), _dev(dst, tuple(dst.shape), "dst"), int(n),
                               _stream(stream)))


def pf_debug_fail_allocs(n: int):
    """Make the library's next ``n`` device allocations fail as out of memory
    (testing aid, include/pf_testing.h)."""
    check(lib().pf_debug_fail_allocs(int(n)))


def pf_version() -> str:
    return lib().pf_version().decode()


def _pf_op(grid: "Grid", o: dict):
    """A ``pf_op`` structure from a dict (keys of :class:`Graph`'s ops) and the
    tensors it refers to."""
    vm = o["vm"]
    ns = _nstate(vm, grid.nb)
    shp = tuple(vm.shape)
    jshp = (grid.nnz_j,) if vm.dim() == 1 else (ns, grid.nnz_j)
    r = PfOp()
    r.op = int(o["op"])
    r.method = int(o.get("method", PF_METHOD_ELEMENTWISE))
    r.nstate = ns
    r.vm = _dev(vm, shp, "vm")
    r.va = _dev(o["va"], shp, "va")
    for name in ("lam_p", "lam_q", "out_a", "out_b"):
        setattr(r, name, _dev(o.get(name), shp, name))
    r.jval = _dev(o.get("jval"), jshp, "jval")
    return r, [v for v in o.values() if not isinstance(v, int)]


def pf_autotune(grid: "Grid", op: dict, cands=None, reps: int = 5):
    """Native schedule autotuner: times candidate schedules of ``op`` (a dict
    as in :class:`Graph`; its outputs are overwritten) and leaves the fastest
    on ``grid``.  ``cands``: (tile_items, states_per_block, order) triples or
    None for the library's default set.  Returns (schedule, us, tried)."""
    r, keep = _pf_op(grid, op)
    c = None if not cands else np.ascontiguousarray(np.asarray(cands, dtype=np.int32).reshape(-1, 3))
    best = np.zeros(3, np.int32)
    us, tried = C.c_double(), C.c_int32()
    check(lib().pf_autotune(grid.handle, C.byref(r), 0 if c is None else len(c), _hp(c), int(reps), _hp(best),
                            C.byref(us), C.byref(tried)))
    del keep
    return (int(best[0]), int(best[1]), int(best[2])), us.value, tried.value


class Graph:
    """Owner of a ``pf_graph`` (pf_graph_create / pf_graph_launch / pf_graph_free).

    ``ops`` is a sequence of dicts with keys ``op`` (PF_OP_*), ``method``,
    ``vm``, ``va`` and, as the op needs them, ``lam_p``, ``lam_q``,
    ``out_a``, ``out_b``, ``jval`` (float64 CUDA tensors; see include/pf.h).
    The graph keeps references to the tensors and to the grid so that they
    outlive it.
    """

    def __init__(self, grid: Grid, ops):
        arr = (PfOp * len(ops))()
        keep = [grid]
        for k, o in enumerate(ops):
            arr[k], kp = _pf_op(grid, o)
            keep += kp
        self._h = C.c_void_p()
        check(lib().pf_graph_create(grid.handle, arr, len(ops), C.byref(self._h)))
        self._keep = keep

    def launch(self, stream=None):
        check(lib().pf_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h and self._h.value:
            lib().pf_graph_free(self._h)
            self._h = C.c_void_p()
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
