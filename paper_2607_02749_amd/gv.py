"""Python binding of ``libgv.so`` (the C ABI in ``include/gv.h``).

Argument marshalling only: every step of the energy and gradient runs in the
library's HIP kernels.  PyTorch supplies device memory (the library borrows
it) and the current HIP stream.  If the library is missing this module raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgv.so")

C64, C128 = 0, 1
ENGINE_FUSED, ENGINE_PLAIN = 0, 1
GRAD_UNCOMPUTE, GRAD_CHECKPOINT, GRAD_RECOMPUTE, GRAD_STORE = 0, 1, 2, 3
ENT_NONE, ENT_CZ_LINEAR, ENT_CZ_CIRCULAR, ENT_CNOT_LINEAR, ENT_CNOT_CIRCULAR = 0, 1, 2, 3, 4
ENT_CNOT_FULL, ENT_CNOT_REVERSE_LINEAR, ENT_CNOT_PAIRWISE, ENT_CNOT_SCA = 5, 6, 7, 8

_PREC = {"c64": C64, "complex64": C64, C64: C64, "c128": C128, "complex128": C128, C128: C128}
_ENGINE = {"fused": ENGINE_FUSED, "plain": ENGINE_PLAIN, ENGINE_FUSED: ENGINE_FUSED,
           ENGINE_PLAIN: ENGINE_PLAIN}
_MODE = {"uncompute": GRAD_UNCOMPUTE, "checkpoint": GRAD_CHECKPOINT, "recompute": GRAD_RECOMPUTE,
         "store": GRAD_STORE, GRAD_UNCOMPUTE: GRAD_UNCOMPUTE, GRAD_CHECKPOINT: GRAD_CHECKPOINT,
         GRAD_RECOMPUTE: GRAD_RECOMPUTE, GRAD_STORE: GRAD_STORE}

ALIGN = 256


class GVError(RuntimeError):
    pass


class _Ansatz(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("layers", ctypes.c_int32), ("ent", ctypes.c_int32),
                ("final_rotation", ctypes.c_int32)]


class _Instance(ctypes.Structure):
    _fields_ = [("ansatz", _Ansatz), ("params_dev", ctypes.c_void_p), ("h", ctypes.c_void_p)]


class _Cluster(ctypes.Structure):
    _fields_ = [("qubit_mask", ctypes.c_uint64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("split_n", ctypes.c_int32), ("lds_n", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library (raises GVError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GVError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_02749_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    AP = ctypes.POINTER(_Ansatz)
    L.gv_version.restype = ctypes.c_char_p
    L.gv_last_error.restype = ctypes.c_char_p
    L.gv_debug_inject_hip_error.argtypes = [i64]
    L.gv_num_params.argtypes = [AP]
    L.gv_num_params.restype = i64
    L.gv_query_sizes.argtypes = [AP, i32, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                 ctypes.POINTER(sz)]
    L.gv_state_create.argtypes = [i32, i32, i32, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]
    L.gv_state_destroy.argtypes = [vp]
    L.gv_state_set_stream.argtypes = [vp, vp]
    L.gv_apply_ansatz.argtypes = [vp, vp, AP]
    L.gv_pauli_sum_create.argtypes = [i32, i64, vp, vp, vp, ctypes.POINTER(vp)]
    L.gv_pauli_sum_destroy.argtypes = [vp]
    L.gv_pauli_sum_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
    L.gv_pauli_sum_device_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.gv_pauli_sum_plan.argtypes = [vp, i32, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
    L.gv_pauli_sum_prepare.argtypes = [vp, vp, vp, sz]
    L.gv_energy.argtypes = [vp, vp, vp]
    L.gv_energy_grad.argtypes = [vp, vp, vp, AP, vp, i32, vp, vp]
    L.gv_pauli_sum_prepare_for.argtypes = [vp, i32, i32, vp, vp, sz]
    IP = ctypes.POINTER(_Instance)
    CP = ctypes.POINTER(_Cluster)
    L.gv_batch_query.argtypes = [i32, IP, i32, ctypes.POINTER(_Tuning), ctypes.POINTER(sz)]
    L.gv_batch_create.argtypes = [i32, IP, CP, i32, ctypes.POINTER(_Tuning), vp, sz, vp, i32,
                                  vp, vp, ctypes.POINTER(vp)]
    L.gv_batch_run.argtypes = [vp]
    L.gv_batch_destroy.argtypes = [vp]
    L.gv_batch_energy_grad.argtypes = [i32, IP, CP, i32, vp, sz, vp, vp, vp]
    L.gv_stream_probe.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, sz, vp]
    L.gv_sample_work_bytes.argtypes = [i32]
    L.gv_sample_work_bytes.restype = sz
    L.gv_sample.argtypes = [i32, i32, vp, vp, i64, vp, sz, vp, vp]
    L.gv_argmax.argtypes = [i32, i32, vp, vp, sz, vp, vp, vp]
    L.gv_pauli_sum_group.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(i64)]
    L.gv_energy_shots_work_bytes.argtypes = [vp, i32, i64]
    L.gv_energy_shots_work_bytes.restype = sz
    L.gv_energy_shots.argtypes = [vp, i32, i32, vp, vp, i64, vp, sz, vp, vp]
    L.gv_profile_enable.argtypes = [vp, i32]
    L.gv_profile_reset.argtypes = [vp]
    L.gv_profile_read.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    for name in ("gv_profile_enable", "gv_profile_reset", "gv_profile_read", "gv_query_sizes",
                 "gv_state_create", "gv_state_destroy", "gv_state_set_stream",
                 "gv_apply_ansatz", "gv_pauli_sum_create", "gv_pauli_sum_destroy",
                 "gv_pauli_sum_info", "gv_pauli_sum_device_bytes", "gv_pauli_sum_prepare",
                 "gv_pauli_sum_prepare_for", "gv_energy", "gv_energy_grad", "gv_batch_query",
                 "gv_batch_create", "gv_batch_run", "gv_batch_destroy", "gv_batch_energy_grad",
                 "gv_stream_probe", "gv_pauli_sum_plan", "gv_sample", "gv_argmax",
                 "gv_pauli_sum_group", "gv_energy_shots"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def inject_hip_error(after: int) -> None:
    """Error-path test hook: the (after+1)-th HIP status check from now
    reports an injected failure (after < 0: off)."""
    _check(lib().gv_debug_inject_hip_error(int(after)), "gv_debug_inject_hip_error")


def _check(status: int, what: str):
    if status != 0:
        raise GVError(f"{what} failed (status {status}): {lib().gv_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _aligned_bytes(nbytes: int, device) -> Tuple[torch.Tensor, torch.Tensor]:
    """A device byte buffer of at least nbytes whose start is ALIGN-aligned;
    returns (owner, aligned view)."""
    nbytes = max(int(nbytes), 1)
    owner = torch.empty(nbytes + ALIGN, dtype=torch.uint8, device=device)
    off = (-owner.data_ptr()) % ALIGN
    return owner, owner[off:off + nbytes]


@dataclass(frozen=True)
class Ansatz:
    """Hardware-efficient ansatz (Sec. IV-B): ``layers`` x [RY all, RZ all,
    entangler], plus one [RY all, RZ all] layer when final_rotation=1."""
    n: int
    layers: int
    ent: int = ENT_CZ_LINEAR
    final_rotation: int = 0

    def c(self) -> _Ansatz:
        return _Ansatz(self.n, self.layers, self.ent, self.final_rotation)

    @property
    def num_params(self) -> int:
        return 2 * self.n * (self.layers + self.final_rotation)


def query_sizes(ansatz: Ansatz, precision="c64", engine="fused", mode="uncompute",
                with_diag=False):
    """(state bytes, work bytes), and the FP64 diagonal's bytes with_diag."""
    a = ansatz.c()
    sb, wb, db = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().gv_query_sizes(ctypes.byref(a), _PREC[precision], _ENGINE[engine], _MODE[mode],
                                ctypes.byref(sb), ctypes.byref(wb), ctypes.byref(db)),
           "gv_query_sizes")
    return (sb.value, wb.value, db.value) if with_diag else (sb.value, wb.value)


STREAM_KINDS = {"read": 0, "write": 1, "copy": 2, "rmw": 3, "triad": 4}


def stream_probe(kind: str, width: int, unroll: int, nontemporal: bool, grid: int,
                 dst: torch.Tensor, src0: Optional[torch.Tensor] = None,
                 src1: Optional[torch.Tensor] = None, nbytes: Optional[int] = None,
                 tile_shift: int = 0):
    """Enqueue one streaming kernel of the bandwidth probe on the current
    stream (see gv_stream_probe in include/gv.h)."""
    nb = dst.numel() * dst.element_size() if nbytes is None else nbytes
    _check(lib().gv_stream_probe(STREAM_KINDS[kind], width, unroll, int(nontemporal), grid,
                                 tile_shift, _ptr(dst), _ptr(src0), _ptr(src1), nb,
                                 _stream_ptr(dst.device)), "gv_stream_probe")


class State:
    """A 2^n-amplitude state in caller (torch) memory plus the workspace the
    gradient sweep needs for ``ansatz`` and ``mode``."""

    def __init__(self, n: int, precision="c64", engine="fused", ansatz: Optional[Ansatz] = None,
                 mode="uncompute", device="cuda", work_bytes: Optional[int] = None):
        self.n = n
        self.precision = _PREC[precision]
        self.engine = _ENGINE[engine]
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        an = ansatz or Ansatz(n, 0)
        sb, wb = query_sizes(an, self.precision, self.engine, mode)
        if work_bytes is not None:
            wb = work_bytes
        self._amps_owner, self.amps = _aligned_bytes(sb, self.device)
        self._work_owner, self.work = _aligned_bytes(wb, self.device)
        self.work_bytes = wb
        h = ctypes.c_void_p()
        _check(lib().gv_state_create(n, self.precision, self.engine, _ptr(self.amps), sb,
                                     _ptr(self.work), wb, _stream_ptr(self.device),
                                     ctypes.byref(h)), "gv_state_create")
        self.handle = h

    def _sync_stream(self):
        lib().gv_state_set_stream(self.handle, _stream_ptr(self.device))

    def amplitudes(self) -> torch.Tensor:
        """The amplitudes as a complex tensor view of the state buffer."""
        real = torch.float32 if self.precision == C64 else torch.float64
        return torch.view_as_complex(self.amps.view(real).view(-1, 2))

    def apply_ansatz(self, theta: torch.Tensor, ansatz: Ansatz):
        assert theta.dtype == torch.float64 and theta.is_contiguous() and theta.device == self.device
        self._sync_stream()
        a = ansatz.c()
        _check(lib().gv_apply_ansatz(self.handle, _ptr(theta), ctypes.byref(a)), "gv_apply_ansatz")

    # per-kernel-class timing (HIP events on the state's stream)
    PROF_KINDS = {"forward_pass": 0, "backward_pass": 1, "energy": 2, "init": 3,
                  "plain_gate": 4, "other": 5, "offdiag": 6, "first_layer": 7,
                  "forward_pass2": 8, "backward_ld": 9, "backward_gf": 10, "backward_gf_ld": 11,
                  "turnaround": 12, "backward2": 13}

    def profile(self, enable: bool = True):
        _check(lib().gv_profile_enable(self.handle, int(enable)), "gv_profile_enable")

    def profile_reset(self):
        _check(lib().gv_profile_reset(self.handle), "gv_profile_reset")

    def profile_read(self) -> dict:
        """{kind: (launches, total ms, total algorithmic bytes)}"""
        out = {}
        for name, k in self.PROF_KINDS.items():
            n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            _check(lib().gv_profile_read(self.handle, k, ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(b)), "gv_profile_read")
            out[name] = (n.value, ms.value, b.value)
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gv_state_destroy(h)
            self.handle = None


class PauliSum:
    """H = sum_k c_k P(x_k, z_k) (Eq. 6); masks are uint64 bit sets."""

    def __init__(self, n: int, x: Sequence[int], z: Sequence[int], c: Sequence[float]):
        self.n = n
        self._x = np.ascontiguousarray(x, dtype=np.uint64)
        self._z = np.ascontiguousarray(z, dtype=np.uint64)
        self._c = np.ascontiguousarray(c, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().gv_pauli_sum_create(n, len(self._c), self._x.ctypes.data, self._z.ctypes.data,
                                         self._c.ctypes.data, ctypes.byref(h)), "gv_pauli_sum_create")
        self.handle = h
        self.device_buffer = None
        self._batches = 0        # live batches built on this Hamiltonian

    def _may_prepare(self):
        if self._batches:
            raise GVError("this PauliSum is used by a live Batch: its device form cannot be "
                          "rebuilt until the batch is gone")

    def info(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gv_pauli_sum_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "gv_pauli_sum_info")
        return a.value, b.value, c.value

    def plan(self, precision="c64", engine="fused") -> Tuple[int, int, int]:
        """(cover passes, most terms in one pass, terms applied one by one)
        for the off-diagonal part on a state of this size (host planning)."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gv_pauli_sum_plan(self.handle, self.n, _PREC[precision], _ENGINE[engine],
                                       ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "gv_pauli_sum_plan")
        return a.value, b.value, c.value

    def prepare(self, state: State):
        self._may_prepare()
        nb = ctypes.c_size_t()
        _check(lib().gv_pauli_sum_device_bytes(self.handle, ctypes.byref(nb)), "device_bytes")
        self._owner, self.device_buffer = _aligned_bytes(nb.value, state.device)
        state._sync_stream()
        _check(lib().gv_pauli_sum_prepare(self.handle, state.handle, _ptr(self.device_buffer),
                                          nb.value), "gv_pauli_sum_prepare")
        return self

    def prepare_for(self, precision="c64", engine="fused", device="cuda"):
        """Device form for states of `precision` on `engine` (and for batches)."""
        self._may_prepare()
        nb = ctypes.c_size_t()
        _check(lib().gv_pauli_sum_device_bytes(self.handle, ctypes.byref(nb)), "device_bytes")
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self._owner, self.device_buffer = _aligned_bytes(nb.value, dev)
        _check(lib().gv_pauli_sum_prepare_for(self.handle, _PREC[precision], _ENGINE[engine],
                                              _stream_ptr(dev), _ptr(self.device_buffer), nb.value),
               "gv_pauli_sum_prepare_for")
        return self

    @property
    def device_bytes(self) -> int:
        """Bytes of the device form (the FP64 diagonal and the off-diagonal tables)."""
        nb = ctypes.c_size_t()
        _check(lib().gv_pauli_sum_device_bytes(self.handle, ctypes.byref(nb)), "device_bytes")
        return nb.value

    def diagonal(self) -> torch.Tensor:
        """The FP64 diagonal of the Z-only part (valid after prepare)."""
        return self.device_buffer[: 8 << self.n].view(torch.float64)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gv_pauli_sum_destroy(h)
            self.handle = None


def energy(state: State, h: PauliSum) -> torch.Tensor:
    """<psi|H|psi> of the state's current psi as float64[2] (re, im)."""
    out = torch.empty(2, dtype=torch.float64, device=state.device)
    state._sync_stream()
    _check(lib().gv_energy(state.handle, h.handle, _ptr(out)), "gv_energy")
    return out


def energy_grad(state: State, h: PauliSum, theta: torch.Tensor, ansatz: Ansatz,
                mask: Optional[torch.Tensor] = None, mode="uncompute",
                out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None):
    """Energy (float64[2]) and gradient (float64[P]) at theta."""
    assert theta.dtype == torch.float64 and theta.is_contiguous() and theta.device == state.device
    if mask is not None:
        assert mask.dtype == torch.uint8 and mask.numel() == ansatz.num_params
    if out is None:
        e = torch.empty(2, dtype=torch.float64, device=state.device)
        g = torch.empty(ansatz.num_params, dtype=torch.float64, device=state.device)
    else:
        e, g = out
    state._sync_stream()
    a = ansatz.c()
    _check(lib().gv_energy_grad(state.handle, h.handle, _ptr(theta), ctypes.byref(a), _ptr(mask),
                                _MODE[mode], _ptr(e), _ptr(g)), "gv_energy_grad")
    return e, g


class GVEnergy(torch.autograd.Function):
    """E(theta) = <psi(theta)|H|psi(theta)> with its gradient from the
    library's reverse sweep.  forward runs energy and gradient in one call
    and keeps the gradient; backward scales it by the incoming gradient."""

    @staticmethod
    def forward(ctx, theta, state: State, h: PauliSum, ansatz: Ansatz,
                mask: Optional[torch.Tensor] = None, mode="uncompute"):
        e, g = energy_grad(state, h, theta.detach().contiguous(), ansatz, mask, mode)
        ctx.save_for_backward(g)
        return e[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None


def param_mask(n: int, layers: int, qubit_mask: int, final_rotation: int = 0,
               device="cuda") -> torch.Tensor:
    """uint8 mask of the RY and RZ parameters of the qubits in qubit_mask, in
    every layer (the block parameter set of Eq. 11)."""
    p = 2 * n * (layers + final_rotation)
    m = torch.zeros(p, dtype=torch.uint8)
    for l in range(layers + final_rotation):
        for g in range(2):
            for q in range(n):
                if (qubit_mask >> q) & 1:
                    m[l * 2 * n + g * n + q] = 1
    return m.to(device)


def _batch_arrays(items, precision, device):
    """ctypes instance and cluster arrays of (Ansatz, theta, PauliSum,
    qubit_mask or None) items; prepares any unprepared Hamiltonian."""
    count = len(items)
    arr = (_Instance * max(count, 1))()
    cl = (_Cluster * max(count, 1))()
    for i, (an, th, h, qmask) in enumerate(items):
        assert th.dtype == torch.float64 and th.is_contiguous() and th.device == device
        assert th.numel() == an.num_params
        if h.device_buffer is None:
            h.prepare_for(precision, "fused", device)
        arr[i].ansatz = an.c()
        arr[i].params_dev = th.data_ptr()
        arr[i].h = h.handle
        cl[i].qubit_mask = ((1 << an.n) - 1) if qmask is None else int(qmask)
    return arr, cl


def _device(device):
    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    return dev


class Batch:
    """Many independent energy + restricted-gradient evaluations in one
    persistent kernel (optionally replayed from a HIP graph) (Sec. IV-D,
    Eq. 11).

    items: sequence of (Ansatz, theta tensor (float64, device), PauliSum,
    qubit_mask or None).  Each PauliSum is prepared here for the batch
    precision if it is not yet.  After run(), energies[i] holds (re, im) and
    grads[i] the gradient of item i (0 outside its qubit block): views of one
    packed buffer, instance i at offset sum_{j<i} P_j.  Rewriting the theta
    tensors in place and calling run() again evaluates the new angles.
    Instances with n >= split_n run as whole-GPU tile passes beside the
    persistent kernel, those with n <= lds_n keep their vectors in LDS (-1:
    never; None: the library defaults).  While the batch lives, its
    PauliSums refuse to be prepared again."""

    def __init__(self, items, precision="c64", blocks_per_cu=None, order=None, graph=True,
                 device="cuda", split_n=None, lds_n=None):
        dev = _device(device)
        self.device = dev
        self.precision = _PREC[precision]
        self.items = list(items)
        count = len(self.items)
        total_p = sum(an.num_params for an, _, _, _ in self.items)
        self.energy_buf = torch.zeros(count, 2, dtype=torch.float64, device=dev)
        self.grad_buf = torch.zeros(max(total_p, 1), dtype=torch.float64, device=dev)
        arr, cl = _batch_arrays(self.items, precision, dev)
        self.grads = []
        off = 0
        for an, _, _, _ in self.items:
            self.grads.append(self.grad_buf[off:off + an.num_params])
            off += an.num_params
        # the Hamiltonians' device buffers must outlive the batch
        self._hams = [h for _, _, h, _ in self.items]
        self._h_buffers = [h._owner for h in self._hams]
        tu = None
        if any(v is not None for v in (blocks_per_cu, order, split_n, lds_n)):
            tu = _Tuning(2 if blocks_per_cu is None else blocks_per_cu, 0 if order is None else order,
                         0 if split_n is None else split_n, 0 if lds_n is None else lds_n)
        self.tuning = tu
        wb = ctypes.c_size_t()
        _check(lib().gv_batch_query(count, arr, self.precision,
                                    None if tu is None else ctypes.byref(tu), ctypes.byref(wb)),
               "gv_batch_query")
        self._work_owner, self.work = _aligned_bytes(wb.value, dev)
        b = ctypes.c_void_p()
        _check(lib().gv_batch_create(count, arr, cl, self.precision,
                                     None if tu is None else ctypes.byref(tu), _ptr(self.work),
                                     wb.value, _stream_ptr(dev), int(graph),
                                     _ptr(self.energy_buf), _ptr(self.grad_buf), ctypes.byref(b)),
               "gv_batch_create")
        self.handle = b
        for h in self._hams:
            h._batches += 1

    @property
    def energies(self) -> torch.Tensor:
        return self.energy_buf

    def run(self):
        _check(lib().gv_batch_run(self.handle), "gv_batch_run")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gv_batch_destroy(h)
            self.handle = None
            for ham in self._hams:
                ham._batches -= 1


def batch_energy_grad(items, precision="c64", device="cuda"):
    """One-shot batch (gv_batch_energy_grad): energies (count x 2) and the
    packed gradients (sum of P_i) of (Ansatz, theta, PauliSum, qubit_mask or
    None) items, enqueued on the current stream."""
    dev = _device(device)
    items = list(items)
    count = len(items)
    arr, cl = _batch_arrays(items, precision, dev)
    total_p = sum(an.num_params for an, _, _, _ in items)
    energies = torch.empty(count, 2, dtype=torch.float64, device=dev)
    grads = torch.empty(max(total_p, 1), dtype=torch.float64, device=dev)
    wb = ctypes.c_size_t()
    _check(lib().gv_batch_query(count, arr, _PREC[precision], None, ctypes.byref(wb)),
           "gv_batch_query")
    owner, work = _aligned_bytes(wb.value, dev)
    _check(lib().gv_batch_energy_grad(count, arr, cl, _PREC[precision], _ptr(work), wb.value,
                                      _stream_ptr(dev), _ptr(energies), _ptr(grads)),
           "gv_batch_energy_grad")
    # `owner` was allocated on the current stream, where the work is queued:
    # torch's caching allocator hands its memory out again only to later work
    # on that stream, so dropping it here is safe
    del owner, work
    return energies, grads


class ParamShift:
    """The parameter-shift gradient of Eq. 13 as one batched launch:
    dE/dtheta_j = (E(theta + pi/2 e_j) - E(theta - pi/2 e_j)) / 2 for every
    j in `indices` (all parameters by default, or a block's P_B of them),
    i.e. 2 |indices| energy-only instances (empty qubit blocks) of one
    ansatz and Hamiltonian, replayed from a HIP graph.  ``__call__(theta)``
    returns (gradient entries at `indices`, the 2 |indices| shifted
    energies)."""

    def __init__(self, ansatz: Ansatz, h: PauliSum, indices=None, precision="c64",
                 device="cuda", graph=True):
        dev = _device(device)
        self.device = dev
        p = ansatz.num_params
        self.indices = np.arange(p) if indices is None else np.asarray(indices, dtype=np.int64)
        m = len(self.indices)
        shift = torch.zeros(2 * m, p, dtype=torch.float64)
        rows = torch.arange(m)
        shift[2 * rows, torch.as_tensor(self.indices)] = np.pi / 2
        shift[2 * rows + 1, torch.as_tensor(self.indices)] = -np.pi / 2
        self.shift = shift.to(dev)
        self.thetas = torch.zeros(2 * m, p, dtype=torch.float64, device=dev)
        items = [(ansatz, self.thetas[i], h, 0) for i in range(2 * m)]
        self.batch = Batch(items, precision, graph=graph, device=dev)

    def __call__(self, theta: torch.Tensor):
        self.thetas.copy_(theta.to(self.device).reshape(1, -1) + self.shift)
        self.batch.run()
        e = self.batch.energies[:, 0]
        return 0.5 * (e[0::2] - e[1::2]), e


# ---------------------------------------------------------------- measurement

def _amps_arg(amps: torch.Tensor):
    """(n, precision code) of a complex64 / complex128 amplitude tensor."""
    assert amps.is_contiguous() and amps.dtype in (torch.complex64, torch.complex128)
    n = amps.numel().bit_length() - 1
    assert amps.numel() == 1 << n
    return n, (C64 if amps.dtype == torch.complex64 else C128)


def sample(amps: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Born-rule indices (uint64 as int64) for the uniform draws u (float64,
    device): inverse-CDF sampling of |amps|^2 (Sec. V-A)."""
    n, prec = _amps_arg(amps)
    assert u.dtype == torch.float64 and u.is_contiguous() and u.device == amps.device
    out = torch.empty(u.numel(), dtype=torch.int64, device=amps.device)
    wb = lib().gv_sample_work_bytes(n)
    owner, work = _aligned_bytes(wb, amps.device)
    _check(lib().gv_sample(n, prec, _ptr(amps), _ptr(u), u.numel(), _ptr(work), wb, _ptr(out),
                           _stream_ptr(amps.device)), "gv_sample")
    return out


def argmax(amps: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """(index, probability) of the most probable basis state (Sec. IV-F)."""
    n, prec = _amps_arg(amps)
    idx = torch.empty(1, dtype=torch.int64, device=amps.device)
    p = torch.empty(1, dtype=torch.float64, device=amps.device)
    wb = lib().gv_sample_work_bytes(n)
    owner, work = _aligned_bytes(wb, amps.device)
    _check(lib().gv_argmax(n, prec, _ptr(amps), _ptr(work), wb, _ptr(idx), _ptr(p),
                           _stream_ptr(amps.device)), "gv_argmax")
    return idx, p


def pauli_groups(h: "PauliSum"):
    """[(X qubits, Y qubits, Z qubits, terms), ...] of the off-diagonal terms."""
    out = []
    _, _, ng = h.info()
    for g in range(ng):
        xm, ym, zm = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        nt = ctypes.c_int64()
        _check(lib().gv_pauli_sum_group(h.handle, g, ctypes.byref(xm), ctypes.byref(ym),
                                        ctypes.byref(zm), ctypes.byref(nt)), "gv_pauli_sum_group")
        out.append((xm.value, ym.value, zm.value, nt.value))
    return out


def energy_shots(h: "PauliSum", amps: torch.Tensor, u: torch.Tensor, shots: int) -> torch.Tensor:
    """The finite-shot energy estimate (Sec. V-A) of the prepared Pauli sum on
    amps; u: (1 + groups) * shots uniform draws (float64, device)."""
    n, prec = _amps_arg(amps)
    assert u.dtype == torch.float64 and u.is_contiguous()
    e = torch.empty(2, dtype=torch.float64, device=amps.device)
    wb = lib().gv_energy_shots_work_bytes(h.handle, prec, shots)
    owner, work = _aligned_bytes(wb, amps.device)
    _check(lib().gv_energy_shots(h.handle, n, prec, _ptr(amps), _ptr(u), shots, _ptr(work), wb,
                                 _ptr(e), _stream_ptr(amps.device)), "gv_energy_shots")
    return e
