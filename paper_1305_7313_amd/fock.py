"""ctypes binding of include/fock.h: argument marshalling only.

Every step of the exchange path runs in libfockx.so.  PyTorch supplies device
memory and the current HIP stream.  Loading fails loudly when the library
has not been built (``python -c "import __graft_entry__ as g; g.build()"``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfockx.so")

FOCK_OK = 0
FOCK_E_ARG = -1
FOCK_E_ALIAS = -2
FOCK_E_SINGULAR_Q = -3
FOCK_E_WORKSPACE = -4
FOCK_E_UNSUPPORTED_GRID = -5
FOCK_E_HIP = -6
FOCK_C128 = 0
FOCK_C64 = 1
FOCK_G0_ZERO = 0
FOCK_G0_GB = 1


class fock_cell(ctypes.Structure):
    _fields_ = [
        ("a", (ctypes.c_double * 3) * 3),
        ("n", ctypes.c_int32 * 3),
        ("npw", ctypes.c_int32),
        ("miller", ctypes.POINTER(ctypes.c_int32)),
        ("ecut_fock", ctypes.c_double),
        ("g0", ctypes.c_int32),
        ("gb_alpha", ctypes.c_double),
        ("nq", ctypes.c_int32 * 3),
    ]


class fock_orbs(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("nb", ctypes.c_int32),
        ("ld", ctypes.c_int32),
    ]


class FockError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status}: {detail}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (paper_1305_7313_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.fock_workspace_size.restype = ctypes.c_size_t
        L.fock_workspace_size.argtypes = [P(fock_cell), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        common = [P(fock_cell), P(ctypes.c_double), ctypes.c_int32, P(fock_orbs), P(fock_orbs)]
        L.fock_apply.restype = ctypes.c_int
        L.fock_apply.argtypes = common + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fock_apply_noalloc.restype = ctypes.c_int
        L.fock_apply_noalloc.argtypes = common + [ctypes.c_void_p, ctypes.c_void_p]
        L.fock_energy.restype = ctypes.c_int
        L.fock_energy.argtypes = common + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fock_energy_backward.restype = ctypes.c_int
        L.fock_energy_backward.argtypes = common + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fock_workspace_size_kmesh.restype = ctypes.c_size_t
        L.fock_workspace_size_kmesh.argtypes = [P(fock_cell), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.fock_energy_kmesh.restype = ctypes.c_int
        L.fock_energy_kmesh.argtypes = [P(fock_cell), ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                                        P(fock_orbs), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]
        L.fock_energy_kmesh_backward.restype = ctypes.c_int
        L.fock_energy_kmesh_backward.argtypes = [P(fock_cell), ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                                                 P(fock_orbs), ctypes.c_void_p, P(ctypes.c_void_p),
                                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fock_energy_kmesh_grad.restype = ctypes.c_int
        L.fock_energy_kmesh_grad.argtypes = [P(fock_cell), ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                                             P(fock_orbs), ctypes.c_void_p, P(ctypes.c_void_p), ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]
        L.fock_batch_plan_create.restype = ctypes.c_int
        L.fock_batch_plan_create.argtypes = [P(fock_cell), P(fock_orbs), P(fock_orbs), P(ctypes.c_double * 3),
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p, P(ctypes.c_void_p)]
        L.fock_batch_apply.restype = ctypes.c_int
        L.fock_batch_apply.argtypes = [ctypes.c_void_p, P(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_void_p]
        L.fock_batch_check.restype = ctypes.c_int
        L.fock_batch_check.argtypes = [ctypes.c_void_p]
        L.fock_batch_set_wait_limit.restype = ctypes.c_int
        L.fock_batch_set_wait_limit.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.fock_batch_plan_info.restype = ctypes.c_char_p
        L.fock_batch_plan_info.argtypes = [ctypes.c_void_p]
        L.fock_batch_plan_destroy.restype = None
        L.fock_batch_plan_destroy.argtypes = [ctypes.c_void_p]
        L.fock_fft3d.restype = ctypes.c_int
        L.fock_fft3d.argtypes = [P(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_void_p]
        L.fock_band_workspace_size.restype = ctypes.c_size_t
        L.fock_band_workspace_size.argtypes = [P(fock_cell), ctypes.c_int32, ctypes.c_int32]
        L.fock_band_density.restype = ctypes.c_int
        L.fock_band_density.argtypes = [P(fock_cell), ctypes.c_int32, P(fock_orbs), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p]
        L.fock_band_force.restype = ctypes.c_int
        L.fock_band_force.argtypes = [P(fock_cell), P(ctypes.c_double), ctypes.c_int32, P(fock_orbs), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.fock_workspace_size_gamma.restype = ctypes.c_size_t
        L.fock_workspace_size_gamma.argtypes = [P(fock_cell), ctypes.c_int32, ctypes.c_int32]
        L.fock_apply_gamma.restype = ctypes.c_int
        L.fock_apply_gamma.argtypes = [P(fock_cell), ctypes.c_int32, P(fock_orbs), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]
        L.fock_exchange_grid.restype = ctypes.c_int
        L.fock_exchange_grid.argtypes = [P(fock_cell), ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                                         P(ctypes.c_int32)]
        L.fock_status_string.restype = ctypes.c_char_p
        L.fock_status_string.argtypes = [ctypes.c_int]
        L.fock_last_error.restype = ctypes.c_char_p
        L.fock_last_error.argtypes = []
        L.fock_trace_enable.restype = ctypes.c_int
        L.fock_trace_enable.argtypes = [ctypes.c_int]
        L.fock_trace_read.restype = ctypes.c_int
        L.fock_trace_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.c_int]
        L.fock_trace_name.restype = ctypes.c_char_p
        L.fock_trace_name.argtypes = [ctypes.c_int]
        L.fock_release_plans.restype = None
        L.fock_release_plans.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != FOCK_OK:
        detail = lib().fock_last_error().decode()
        raise FockError(status, f"{lib().fock_status_string(status).decode()}: {detail}")


class Cell:
    """Host description of the cell, grid and sphere (keeps the Miller array alive)."""

    def __init__(self, a, n, miller, ecut_fock: float = 0.0, g0: int = FOCK_G0_ZERO,
                 gb_alpha: float = 0.0, nq=(1, 1, 1)):
        self.a = np.ascontiguousarray(a, dtype=np.float64).reshape(3, 3)
        self.n = tuple(int(x) for x in n)
        self.miller = np.ascontiguousarray(miller, dtype=np.int32).reshape(-1, 3)
        self.ecut_fock = float(ecut_fock)
        self.g0 = int(g0)
        self.gb_alpha = float(gb_alpha)
        self.nq = tuple(int(x) for x in nq)
        c = fock_cell()
        for i in range(3):
            for j in range(3):
                c.a[i][j] = float(self.a[i, j])
            c.n[i] = self.n[i]
            c.nq[i] = self.nq[i]
        c.npw = int(self.miller.shape[0])
        c.miller = self.miller.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        c.ecut_fock = self.ecut_fock
        c.g0 = self.g0
        c.gb_alpha = self.gb_alpha
        self.c = c

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])


def dtype_code(t) -> int:
    import torch
    if t.dtype == torch.complex128:
        return FOCK_C128
    if t.dtype == torch.complex64:
        return FOCK_C64
    raise TypeError(f"orbital coefficients must be complex128 or complex64, not {t.dtype}")


def _like(t, ref, name):
    """t must hold ref's dtype on ref's device: the library reads and writes
    every complex array of a call at the element size of one dtype."""
    if t.dtype != ref.dtype:
        raise ValueError(f"{name} is {t.dtype}; every coefficient, output and gradient of this call must be "
                         f"{ref.dtype}")
    if t.device != ref.device:
        raise ValueError(f"{name} is on {t.device}, not on {ref.device}")


def _rows(t, ref, name, nb, npw, ld=None):
    """t: [>= nb, >= npw] rows of ref's dtype and device, unit stride along G,
    and (with more than one row) the leading dimension ld the library uses."""
    _like(t, ref, name)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be [nb, npw] with unit stride along G")
    if t.shape[0] < nb or t.shape[1] < npw:
        raise ValueError(f"{name} is {tuple(t.shape)}, smaller than [{nb}, {npw}]")
    if ld is not None and nb > 1 and t.stride(0) != ld:
        raise ValueError(f"{name} must have the leading dimension {ld} of its coefficient block")


def orbs(c, w, npw=None) -> fock_orbs:
    """fock_orbs over a device tensor c [nb, ld] (row-major) and weights w [nb]
    (float64, on c's device); npw: the sphere size every row must hold."""
    import torch
    if c.dim() != 2 or c.stride(1) != 1:
        raise ValueError("coefficients must be [nb, ld] with unit stride along G")
    if npw is not None and c.shape[0] > 0 and c.shape[1] < npw:
        raise ValueError(f"coefficients hold {c.shape[1]} plane waves per row, fewer than the sphere's {npw}")
    if w.dtype != torch.float64 or not w.is_contiguous():
        raise ValueError("weights must be a contiguous float64 tensor")
    if w.device != c.device:
        raise ValueError(f"weights are on {w.device}, the coefficients on {c.device}")
    if w.numel() != c.shape[0]:
        raise ValueError("one weight per orbital")
    o = fock_orbs()
    o.c = c.data_ptr() if c.numel() else None
    o.w = w.data_ptr() if w.numel() else None
    o.nb = int(c.shape[0])
    o.ld = int(c.stride(0)) if c.shape[0] > 1 else int(c.shape[1])
    return o


def _stream(device=None):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _qarr(q):
    return (ctypes.c_double * 3)(*[float(x) for x in q])


def fock_apply_gamma(cell: Cell, c, f, out=None, ws=None):
    """V_x of a block of real (Gamma) orbitals applied to itself: [nb, npw]
    (C call: fock_apply_gamma; c must hold c(-G) = conj(c(G)))."""
    import torch
    dt = dtype_code(c)
    o = orbs(c, f, cell.npw)
    if out is None:
        out = torch.empty((c.shape[0], cell.npw), dtype=c.dtype, device=c.device)
    _rows(out, c, "out", o.nb, cell.npw, o.ld)
    if ws is None:
        nbytes = int(lib().fock_workspace_size_gamma(ctypes.byref(cell.c), dt, o.nb))
        if nbytes == 0:
            raise FockError(FOCK_E_UNSUPPORTED_GRID, "fock_workspace_size_gamma returned 0 for this cell")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=c.device)
    _check(lib().fock_apply_gamma(ctypes.byref(cell.c), dt, ctypes.byref(o), out.data_ptr() if out.numel() else None,
                                  ws.data_ptr(), ws.numel(), _stream(c.device)))
    return out


def band_workspace(cell: Cell, dtype: int, nb: int, device):
    import torch
    nbytes = int(lib().fock_band_workspace_size(ctypes.byref(cell.c), int(dtype), int(nb)))
    if nbytes == 0:
        raise FockError(FOCK_E_UNSUPPORTED_GRID, "fock_band_workspace_size returned 0 for this cell")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def fock_band_density(cell: Cell, c, w, out=None, ws=None):
    """Charge density sum_b w_b |psi_b(r)|^2 on the grid: float64 [n1, n2, n3]
    (C call: fock_band_density)."""
    import torch
    dt = dtype_code(c)
    o = orbs(c, w, cell.npw)
    if out is None:
        out = torch.empty(cell.n, dtype=torch.float64, device=c.device)
    if out.dtype != torch.float64 or out.device != c.device or not out.is_contiguous() or tuple(out.shape) != cell.n:
        raise ValueError("out must be a contiguous float64 [n1, n2, n3] tensor on the orbitals' device")
    if ws is None:
        ws = band_workspace(cell, dt, o.nb, c.device)
    _check(lib().fock_band_density(ctypes.byref(cell.c), dt, ctypes.byref(o), out.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream(c.device)))
    return out


def fock_band_force(cell: Cell, k, c, w, vloc, out=None, ws=None):
    """-w_b (1/2 |k+G|^2 c_b + (V psi_b)(G)) on the sphere: [nb, npw] of c's dtype;
    vloc is real [n1, n2, n3] in c's precision (C call: fock_band_force)."""
    import torch
    dt = dtype_code(c)
    rdt = torch.float64 if dt == FOCK_C128 else torch.float32
    if vloc.dtype != rdt or not vloc.is_contiguous() or tuple(vloc.shape) != cell.n or vloc.device != c.device:
        raise ValueError("vloc must be a contiguous real [n1, n2, n3] tensor in the orbitals' precision and device")
    o = orbs(c, w, cell.npw)
    if out is None:
        out = torch.empty_like(c)
    _like(out, c, "out")
    if out.shape != c.shape or out.stride() != c.stride():
        raise ValueError("out must have the coefficients' shape and strides")
    if ws is None:
        ws = band_workspace(cell, dt, o.nb, c.device)
    _check(lib().fock_band_force(ctypes.byref(cell.c), _qarr(k), dt, ctypes.byref(o), vloc.data_ptr(),
                                 out.data_ptr() if out.numel() else None, ws.data_ptr(), ws.numel(),
                                 _stream(c.device)))
    return out


def fock_exchange_grid(cell: Cell, q=None, dtype: int = FOCK_C128) -> tuple:
    """Compiled grid of fewest points on which this sphere and cell.ecut_fock
    give grid-independent results for every q in q ([nq, 3]; None: q = 0)
    (C call: fock_exchange_grid; cell.n is not read)."""
    qs = np.zeros((0, 3)) if q is None else np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    qp = qs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(qs) else None
    out = (ctypes.c_int32 * 3)()
    _check(lib().fock_exchange_grid(ctypes.byref(cell.c), len(qs), qp, int(dtype), out))
    return tuple(int(x) for x in out)


def fock_workspace_size(cell: Cell, dtype: int, n_occ: int, n_tgt: int) -> int:
    return int(lib().fock_workspace_size(ctypes.byref(cell.c), int(dtype), int(n_occ), int(n_tgt)))


def workspace(cell: Cell, dtype: int, n_occ: int, n_tgt: int, device):
    import torch
    nbytes = fock_workspace_size(cell, dtype, n_occ, n_tgt)
    if nbytes == 0:
        raise FockError(FOCK_E_UNSUPPORTED_GRID, "fock_workspace_size returned 0 for this cell")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def fock_apply(cell: Cell, q, c_occ, f_occ, c_tgt, out=None, ws=None):
    """(V_x psi_j) on the sphere for every target: a [n_tgt, npw] tensor (C call: fock_apply)."""
    import torch
    dt = dtype_code(c_occ)
    _like(c_tgt, c_occ, "c_tgt")
    if out is not None:
        _like(out, c_occ, "out")
    ones = torch.ones(c_tgt.shape[0], dtype=torch.float64, device=c_tgt.device)
    o, t = orbs(c_occ, f_occ, cell.npw), orbs(c_tgt, ones, cell.npw)
    if out is None:
        out = torch.empty((c_tgt.shape[0], cell.npw), dtype=c_tgt.dtype, device=c_tgt.device)
    _rows(out, c_occ, "out", t.nb, cell.npw, t.ld)
    if ws is None:
        ws = workspace(cell, dt, o.nb, t.nb, c_occ.device)
    _check(lib().fock_apply(ctypes.byref(cell.c), _qarr(q), dt, ctypes.byref(o), ctypes.byref(t),
                            out.data_ptr() if out.numel() else None, ws.data_ptr(), ws.numel(),
                            _stream(c_occ.device)))
    return out


NOALLOC_SCRATCH_BYTES = 32 << 20  # FOCK_NOALLOC_SCRATCH_BYTES of include/fock.h


def fock_apply_noalloc(cell: Cell, q, c_occ, f_occ, c_tgt, out):
    """fock_apply without a workspace: the library uses its fixed per-GPU
    scratch array and allocates nothing (C call: fock_apply_noalloc).  out is
    the caller's [n_tgt, npw] result tensor."""
    import torch
    _like(c_tgt, c_occ, "c_tgt")
    ones = torch.ones(c_tgt.shape[0], dtype=torch.float64, device=c_tgt.device)
    o, t = orbs(c_occ, f_occ, cell.npw), orbs(c_tgt, ones, cell.npw)
    _rows(out, c_occ, "out", t.nb, cell.npw, t.ld)
    _check(lib().fock_apply_noalloc(ctypes.byref(cell.c), _qarr(q), dtype_code(c_occ), ctypes.byref(o),
                                    ctypes.byref(t), out.data_ptr() if out.numel() else None,
                                    _stream(c_occ.device)))
    return out


def fock_energy(cell: Cell, q, c_occ, f_occ, c_tgt, g_tgt, out=None, ws=None):
    """Exchange energy as a device float64 scalar tensor (C call: fock_energy)."""
    import torch
    dt = dtype_code(c_occ)
    _like(c_tgt, c_occ, "c_tgt")
    o, t = orbs(c_occ, f_occ, cell.npw), orbs(c_tgt, g_tgt, cell.npw)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=c_occ.device)
    if out.dtype != torch.float64 or out.device != c_occ.device or out.numel() < 1:
        raise ValueError("out must be a float64 scalar on the coefficients' device")
    if ws is None:
        ws = workspace(cell, dt, o.nb, t.nb, c_occ.device)
    _check(lib().fock_energy(ctypes.byref(cell.c), _qarr(q), dt, ctypes.byref(o), ctypes.byref(t),
                             out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(c_occ.device)))
    return out


def fock_energy_backward(cell: Cell, q, c_occ, f_occ, c_tgt, g_tgt, grad_ex, grad_occ=None, grad_tgt=None,
                         ws=None):
    """Wirtinger gradients grad_ex * dE/dconj(c) into grad_occ / grad_tgt (C call: fock_energy_backward)."""
    import torch
    dt = dtype_code(c_occ)
    _like(c_tgt, c_occ, "c_tgt")
    o, t = orbs(c_occ, f_occ, cell.npw), orbs(c_tgt, g_tgt, cell.npw)
    if grad_ex.dtype != torch.float64 or grad_ex.device != c_occ.device or grad_ex.numel() < 1:
        raise ValueError("grad_ex must be a float64 scalar on the coefficients' device")
    if grad_occ is not None:
        _rows(grad_occ, c_occ, "grad_occ", o.nb, cell.npw, o.ld)
    if grad_tgt is not None:
        _rows(grad_tgt, c_occ, "grad_tgt", t.nb, cell.npw, t.ld)
    if ws is None:
        ws = workspace(cell, dt, o.nb, t.nb, c_occ.device)
    _check(lib().fock_energy_backward(
        ctypes.byref(cell.c), _qarr(q), dt, ctypes.byref(o), ctypes.byref(t), grad_ex.data_ptr(),
        grad_occ.data_ptr() if grad_occ is not None and grad_occ.numel() else None,
        grad_tgt.data_ptr() if grad_tgt is not None and grad_tgt.numel() else None,
        ws.data_ptr(), ws.numel(), _stream(c_occ.device)))
    return grad_occ, grad_tgt


def fock_fft3d(x, sign: int):
    """In-place unnormalised 3-D transform of x [nb, n1, n2, n3] (C call: fock_fft3d)."""
    n = (ctypes.c_int32 * 3)(*x.shape[-3:])
    nb = int(np.prod(x.shape[:-3])) if x.dim() > 3 else 1
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    _check(lib().fock_fft3d(n, dtype_code(x), int(sign), x.data_ptr(), nb, _stream(x.device)))
    return x


def fock_release_plans():
    lib().fock_release_plans()


def fock_trace_enable(on: bool) -> int:
    return int(lib().fock_trace_enable(1 if on else 0))


def fock_trace_read(reset: bool = True) -> dict:
    """{kernel class: (milliseconds, launches)} accumulated since the last reset."""
    n = int(lib().fock_trace_read(None, None, 0))
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    lib().fock_trace_read(ms, cnt, 1 if reset else 0)
    return {lib().fock_trace_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(n)}


# ---------------------------------------------------------------------------
# k-point mesh
# ---------------------------------------------------------------------------
def _kmesh_args(cell, kpts, C, W):
    if C.dim() != 3 or W.dim() != 2 or tuple(W.shape) != tuple(C.shape[:2]):
        raise ValueError("C must be [nk, nb, npw] and W [nk, nb]")
    nk = int(C.shape[0])
    kp = np.ascontiguousarray(np.asarray(kpts, dtype=np.float64).reshape(nk, 3))
    sets = (fock_orbs * nk)()
    for k in range(nk):
        sets[k] = orbs(C[k], W[k], cell.npw)
    return nk, kp, sets


def _scalar_out(out, C, name="out"):
    import torch
    if out.dtype != torch.float64 or out.device != C.device or out.numel() < 1:
        raise ValueError(f"{name} must be a float64 scalar on the coefficients' device")


def fock_workspace_size_kmesh(cell: Cell, dtype: int, nk: int, nb_max: int) -> int:
    return int(lib().fock_workspace_size_kmesh(ctypes.byref(cell.c), int(dtype), int(nk), int(nb_max)))


def workspace_kmesh(cell: Cell, dtype: int, nk: int, nb_max: int, device):
    import torch
    nbytes = fock_workspace_size_kmesh(cell, dtype, nk, nb_max)
    if nbytes == 0:
        raise FockError(FOCK_E_UNSUPPORTED_GRID, "fock_workspace_size_kmesh returned 0 for this cell")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def fock_energy_kmesh(cell: Cell, kpts, C, W, out=None, ws=None):
    """Exchange energy over a k-mesh: C [nk, nb, npw] device coefficients, W [nk, nb] float64
    weights (occupation / N_k).  Returns a device float64 scalar (C call: fock_energy_kmesh)."""
    import torch
    dt = dtype_code(C)
    nk, kp, sets = _kmesh_args(cell, kpts, C, W)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=C.device)
    _scalar_out(out, C)
    if ws is None:
        ws = workspace_kmesh(cell, dt, nk, int(C.shape[1]), C.device)
    _check(lib().fock_energy_kmesh(ctypes.byref(cell.c), nk, kp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   dt, sets, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(C.device)))
    return out


def fock_energy_kmesh_backward(cell: Cell, kpts, C, W, grad_ex, grad, ws=None):
    """grad[k] = grad_ex * dE/dconj(C[k]) (C call: fock_energy_kmesh_backward);
    a None entry skips that k-point."""
    dt = dtype_code(C)
    nk, kp, sets = _kmesh_args(cell, kpts, C, W)
    _scalar_out(grad_ex, C, "grad_ex")
    if len(grad) != nk:
        raise ValueError("one gradient entry (or None) per k-point")
    for k in range(nk):
        if grad[k] is not None:
            _rows(grad[k], C, f"grad[{k}]", sets[k].nb, cell.npw, sets[k].ld)
    ptrs = (ctypes.c_void_p * nk)(*[grad[k].data_ptr() if grad[k] is not None else None for k in range(nk)])
    if ws is None:
        ws = workspace_kmesh(cell, dt, nk, int(C.shape[1]), C.device)
    _check(lib().fock_energy_kmesh_backward(ctypes.byref(cell.c), nk,
                                            kp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dt, sets,
                                            grad_ex.data_ptr(), ptrs, ws.data_ptr(), ws.numel(),
                                            _stream(C.device)))
    return grad


def fock_energy_kmesh_grad(cell: Cell, kpts, C, W, grad=None, out=None, ws=None):
    """E and grad[k] = dE/dconj(C[k]) from one pass (C call:
    fock_energy_kmesh_grad).  Returns (E as a device FP64 scalar, grad)."""
    import torch
    dt = dtype_code(C)
    nk, kp, sets = _kmesh_args(cell, kpts, C, W)
    if grad is None:
        grad = torch.empty_like(C)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=C.device)
    _scalar_out(out, C)
    if len(grad) != nk:
        raise ValueError("one gradient block per k-point")
    for k in range(nk):
        _rows(grad[k], C, f"grad[{k}]", sets[k].nb, cell.npw, sets[k].ld)
    ptrs = (ctypes.c_void_p * nk)(*[grad[k].data_ptr() for k in range(nk)])
    if ws is None:
        ws = workspace_kmesh(cell, dt, nk, int(C.shape[1]), C.device)
    _check(lib().fock_energy_kmesh_grad(ctypes.byref(cell.c), nk,
                                        kp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dt, sets,
                                        out.data_ptr(), ptrs, ws.data_ptr(), ws.numel(), _stream(C.device)))
    return out, grad


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
class BatchPlan:
    """Several systems, each an apply as fock_apply (occupied block, target
    block, q), in one hipGraph (C calls: fock_batch_plan_create / _apply /
    _check / _plan_info / _plan_destroy).  tgt_coeffs None: each block is
    applied to itself; q None: q = 0.  The tensors passed here are bound to
    the graph and must stay alive; apply() fills self.outs and self.ex."""

    def __init__(self, cells, coeffs, weights, tgt_coeffs=None, tgt_weights=None, q=None, tune_cache=None):
        import torch
        n = len(cells)
        if not (len(coeffs) == len(weights) == n):
            raise ValueError("one coefficient block and one weight vector per cell")
        if (tgt_coeffs is None) != (tgt_weights is None):
            raise ValueError("target coefficients and weights go together")
        if n == 0:
            raise ValueError("a batch needs at least one system")
        dt = dtype_code(coeffs[0])
        self.cells, self.coeffs, self.weights = list(cells), list(coeffs), list(weights)
        self.tgt_coeffs = list(tgt_coeffs) if tgt_coeffs is not None else self.coeffs
        self.tgt_weights = list(tgt_weights) if tgt_weights is not None else self.weights
        if not (len(self.tgt_coeffs) == len(self.tgt_weights) == n):
            raise ValueError("one target block and one target weight vector per cell")
        if q is not None and len(q) != n:
            raise ValueError("one q-vector per cell")
        ref = coeffs[0]
        for k in range(n):
            _like(self.coeffs[k], ref, f"coeffs[{k}]")
            _like(self.tgt_coeffs[k], ref, f"tgt_coeffs[{k}]")
            orbs(self.coeffs[k], self.weights[k], self.cells[k].npw)
            orbs(self.tgt_coeffs[k], self.tgt_weights[k], self.cells[k].npw)
        self.outs = [torch.empty_like(c) for c in self.tgt_coeffs]
        self.ex = torch.empty(n, dtype=torch.float64, device=coeffs[0].device)
        cs = (fock_cell * n)(*[c.c for c in self.cells])
        occ = (fock_orbs * n)(*[orbs(c, w) for c, w in zip(self.coeffs, self.weights)])
        tgt = None
        if tgt_coeffs is not None:
            tgt = (fock_orbs * n)(*[orbs(c, w) for c, w in zip(self.tgt_coeffs, self.tgt_weights)])
        qa = None
        if q is not None:
            q3 = ctypes.c_double * 3
            qa = (q3 * n)(*[q3(*[float(x) for x in qq]) for qq in q])
        plan = ctypes.c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        _check(lib().fock_batch_plan_create(cs, occ, tgt, qa, n, dt, cache, ctypes.byref(plan)))
        self._plan = plan
        self._outp = (ctypes.c_void_p * n)(*[o.data_ptr() if o.numel() else None for o in self.outs])

    def apply(self, stream=None):
        import torch
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream) if stream is None else stream
        _check(lib().fock_batch_apply(self._plan, self._outp, self.ex.data_ptr(), s))
        return self.outs

    def check(self):
        _check(lib().fock_batch_check(self._plan))

    def set_wait_limit(self, ms: float):
        """Bound on one dependency wait of the persistent kernel, in ms (<= 0: the plan's default)."""
        _check(lib().fock_batch_set_wait_limit(self._plan, float(ms)))

    def info(self) -> dict:
        import json
        return json.loads(lib().fock_batch_plan_info(self._plan).decode())

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib().fock_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
