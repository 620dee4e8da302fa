"""Python binding of the C ABI in include/gkr.h (argument marshalling only).

Every step of proving runs in libgkr.so; this module converts arguments,
allocates caller-owned device buffers through torch and checks status codes.
If the library has not been built the import fails loudly: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgkr.so")

GKR_OK = 0
GKR_EINVAL = -1
GKR_ENOMEM = -2
GKR_EDEVICE = -3
GKR_EBUFSZ = -4
GKR_EUNSUPPORTED = -5

# Every symbol include/gkr.h declares.
EXPORTS = (
    "gkr_last_error", "gkr_circuit_create", "gkr_circuit_destroy", "gkr_workspace_bytes",
    "gkr_proof_bytes", "gkr_layer_proof_bytes", "gkr_gate_layers", "gkr_prove_circuit",
    "gkr_transcript_init", "gkr_output_claim", "gkr_prove_layer", "gkr_verify",
    "gkr_plan_create", "gkr_plan_destroy", "gkr_plan_reset", "gkr_run_batch", "gkr_plan_progress",
    "gkr_prove_batch", "gkr_set_tuning", "gkr_get_tuning", "gkr_profile_enable", "gkr_profile_read",
    "gkr_ubench", "gkr_prove_circuit_noalloc", "gkr_general_circuit_create", "gkr_circuit_create_field",
    "gkr_gl_prove_circuit", "gkr_gl_verify",
)

FIELD_BN254 = 0
FIELD_GOLDILOCKS = 1
GOLDILOCKS_P = (1 << 64) - (1 << 32) + 1

# Size of the static workspace of gkr_prove_circuit_noalloc (GKR_NOALLOC_WORKSPACE_BYTES).
NOALLOC_WORKSPACE_BYTES = 256 << 20


class GkrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("gkr error %d: %s" % (code, msg))
        self.code = code


class Gate(ctypes.Structure):
    """gkr_gate: x, y (u32), type (u8), three reserved bytes. A (count, 3)
    uint32 array with the type in the third word has this layout (little
    endian, type < 256)."""
    _fields_ = [("x", ctypes.c_uint32), ("y", ctypes.c_uint32), ("type", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8 * 3)]


class NestedGate(ctypes.Structure):
    """gkr_nested_gate: z, x, src, y (u32), type (u8), three reserved bytes. A
    (count, 5) uint32 array with the type in the fifth word has this layout."""
    _fields_ = [("z", ctypes.c_uint32), ("x", ctypes.c_uint32), ("src", ctypes.c_uint32), ("y", ctypes.c_uint32),
                ("type", ctypes.c_uint8), ("reserved", ctypes.c_uint8 * 3)]


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgkr.so is not built; run __graft_entry__.build() "
                              "or python -m paper_2404_10404_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.gkr_last_error.restype = ctypes.c_char_p
        L.gkr_circuit_create.argtypes = [_u32, _u32, ctypes.POINTER(_u32), ctypes.POINTER(ctypes.POINTER(Gate)),
                                         ctypes.POINTER(_vp)]
        L.gkr_circuit_create.restype = _i32
        L.gkr_general_circuit_create.argtypes = [_u32, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_u64),
                                                 ctypes.POINTER(ctypes.POINTER(NestedGate)), ctypes.POINTER(_vp)]
        L.gkr_general_circuit_create.restype = _i32
        L.gkr_circuit_create_field.argtypes = [_u32, _u32, _u32, ctypes.POINTER(_u32),
                                               ctypes.POINTER(ctypes.POINTER(Gate)), ctypes.POINTER(_vp)]
        L.gkr_circuit_create_field.restype = _i32
        L.gkr_gl_prove_circuit.argtypes = [_vp, _vp, _u64, _vp, _vp, _sz, ctypes.POINTER(_sz), _vp, _sz, _vp]
        L.gkr_gl_prove_circuit.restype = _i32
        L.gkr_gl_verify.argtypes = [_vp, _vp, _vp, _u64, _vp, _sz]
        L.gkr_gl_verify.restype = _i32
        L.gkr_circuit_destroy.argtypes = [_vp]
        L.gkr_circuit_destroy.restype = None
        for name in ("gkr_workspace_bytes", "gkr_proof_bytes"):
            getattr(L, name).argtypes = [_vp]
            getattr(L, name).restype = _sz
        L.gkr_layer_proof_bytes.argtypes = [_vp, _u32]
        L.gkr_layer_proof_bytes.restype = _sz
        L.gkr_gate_layers.argtypes = [_vp]
        L.gkr_gate_layers.restype = _u64
        L.gkr_prove_circuit.argtypes = [_vp, _vp, _u64, _vp, _vp, _sz, ctypes.POINTER(_sz), _vp, _sz, _vp]
        L.gkr_prove_circuit.restype = _i32
        L.gkr_transcript_init.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.gkr_transcript_init.restype = _i32
        L.gkr_output_claim.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.gkr_output_claim.restype = _i32
        L.gkr_prove_layer.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _sz, _vp]
        L.gkr_prove_layer.restype = _i32
        L.gkr_verify.argtypes = [_vp, _vp, _vp, _u64, _vp, _sz]
        L.gkr_verify.restype = _i32
        L.gkr_set_tuning.argtypes = [_u32, _u32, _u32]
        L.gkr_set_tuning.restype = _i32
        L.gkr_prove_circuit_noalloc.argtypes = [_vp, _vp, _u64, _vp, _vp, _sz, ctypes.POINTER(_sz), _vp]
        L.gkr_prove_circuit_noalloc.restype = _i32
        L.gkr_ubench.argtypes = [_u32, _u32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.gkr_ubench.restype = _i32
        L.gkr_committed_sizes.argtypes = [_vp, _u32, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]
        L.gkr_committed_sizes.restype = _i32
        L.gkr_prove_circuit_committed.argtypes = [_vp, _vp, _u64, _u32, _vp, _vp, _sz, _vp, _sz, _vp]
        L.gkr_prove_circuit_committed.restype = _i32
        L.gkr_verify_committed.argtypes = [_vp, _vp, _u64, _u32, _vp, _sz]
        L.gkr_verify_committed.restype = _i32
        L.gkr_vpd_workspace_bytes.argtypes = [_u32, ctypes.POINTER(_sz)]
        L.gkr_vpd_workspace_bytes.restype = _i32
        L.gkr_vpd_commit.argtypes = [_u32, _vp, _vp, _vp, _sz, _vp]
        L.gkr_vpd_commit.restype = _i32
        _lib = L
        _apply_tuning_cache(L)
    return _lib


TUNING_CACHE = os.path.join(_HERE, "tuning.json")
_tuned = {}


def _apply_tuning_cache(L):
    """Apply the autotuner's cached choice (paper_2404_10404_amd/autotune.py), if present."""
    if not os.path.exists(TUNING_CACHE):
        return
    import json
    with open(TUNING_CACHE) as f:
        best = json.load(f).get("best", {})
    if "tail_log" in best and "max_round_blocks" in best:
        _check_with(L, L.gkr_set_tuning(int(best["tail_log"]), int(best["max_round_blocks"]),
                                        int(best.get("pairs_per_thread", 1))))
    _tuned.update(best)


def _check_with(L, rc):
    if rc < 0:
        raise GkrError(rc, L.gkr_last_error().decode())


def tuned_batch_workgroups() -> int:
    """Resident workgroups of the batch kernel chosen by the autotuner (0 = fill the device)."""
    lib()
    return int(_tuned.get("batch_workgroups", 0))


def _check(rc: int) -> int:
    if rc < 0:
        raise GkrError(rc, lib().gkr_last_error().decode())
    return rc


def _elements(arr) -> np.ndarray:
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    if a.ndim != 2 or a.shape[1] != 8:
        raise ValueError("elements must have shape (count, 8)")
    return a


class Circuit:
    """A circuit object of the library (wiring uploaded to the current device).
    field: FIELD_BN254 (gkr_circuit_create) or FIELD_GOLDILOCKS."""

    def __init__(self, depth: int, log_copies: int, log_sub_width: Sequence[int],
                 wiring: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]], field: int = FIELD_BN254):
        L = lib()
        self.depth, self.log_copies = int(depth), int(log_copies)
        self.log_sub_width = [int(s) for s in log_sub_width]
        sig = (_u32 * len(self.log_sub_width))(*self.log_sub_width)
        self._gate_arrays = []
        ptrs = (ctypes.POINTER(Gate) * max(1, len(wiring)))()
        for i, (x, y, t) in enumerate(wiring):
            g = np.empty((len(x), 3), dtype=np.uint32)
            g[:, 0], g[:, 1], g[:, 2] = x, y, t
            self._gate_arrays.append(g)
            ptrs[i] = g.ctypes.data_as(ctypes.POINTER(Gate))
        h = _vp()
        self.field = int(field)
        if self.field == FIELD_BN254:
            _check(L.gkr_circuit_create(self.depth, self.log_copies, sig, ptrs, ctypes.byref(h)))
        else:
            _check(L.gkr_circuit_create_field(self.field, self.depth, self.log_copies, sig, ptrs, ctypes.byref(h)))
        self._h = h
        self._gate_arrays = None

    @classmethod
    def from_synth(cls, spec, wiring, field: int = FIELD_BN254) -> "Circuit":
        return cls(spec.depth, spec.log_copies, spec.log_sub_width, [(w.x, w.y, w.kind) for w in wiring], field)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gkr_circuit_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def s(self, i: int) -> int:
        return self.log_sub_width[i] + self.log_copies

    @property
    def workspace_bytes(self) -> int:
        return lib().gkr_workspace_bytes(self._h)

    @property
    def proof_bytes(self) -> int:
        return lib().gkr_proof_bytes(self._h)

    def layer_proof_bytes(self, layer: int) -> int:
        return lib().gkr_layer_proof_bytes(self._h, layer)

    @property
    def gate_layers(self) -> int:
        return lib().gkr_gate_layers(self._h)


class GeneralCircuit(Circuit):
    """A general circuit (nested gates with right inputs from any later layer)."""

    def __init__(self, depth: int, log_copies: int, log_sub_width: Sequence[int],
                 layers: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray, np.ndarray]]):
        L = lib()
        self.depth, self.log_copies = int(depth), int(log_copies)
        self.log_sub_width = [int(s) for s in log_sub_width]
        sig = (_u32 * len(self.log_sub_width))(*self.log_sub_width)
        arrays = []
        counts = (_u64 * max(1, len(layers)))()
        ptrs = (ctypes.POINTER(NestedGate) * max(1, len(layers)))()
        for i, (z, x, src, y, t) in enumerate(layers):
            g = np.empty((len(z), 5), dtype=np.uint32)
            g[:, 0], g[:, 1], g[:, 2], g[:, 3], g[:, 4] = z, x, src, y, t
            arrays.append(g)
            counts[i] = len(z)
            ptrs[i] = g.ctypes.data_as(ctypes.POINTER(NestedGate))
        h = _vp()
        _check(L.gkr_general_circuit_create(self.depth, self.log_copies, sig, counts, ptrs, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_synth(cls, spec, wiring) -> "GeneralCircuit":
        return cls(spec.depth, spec.log_copies, spec.log_sub_width,
                   [(w.z, w.x, w.src, w.y, w.kind) for w in wiring])


# ------------------------------------------------------------ device-level calls

def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def device_elements(arr, device="cuda"):
    """Upload (count, 8) uint32 canonical elements as a torch int32 tensor."""
    import torch
    a = _elements(arr)
    return torch.from_numpy(a.view(np.int32)).to(device)


def host_elements(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32).reshape(-1, 8)


def alloc_bytes(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(1, (nbytes + 255) // 256 * 256), dtype=torch.uint8, device=device)


def prove_circuit(c: Circuit, d_inputs, seed: int, d_outputs, d_proof, d_ws, stream=None) -> int:
    """gkr_prove_circuit on caller tensors; returns the proof length."""
    plen = _sz(0)
    _check(lib().gkr_prove_circuit(c.handle, _ptr(d_inputs), seed & (2**64 - 1), _ptr(d_outputs), _ptr(d_proof),
                                   d_proof.numel() * d_proof.element_size(), ctypes.byref(plen), _ptr(d_ws),
                                   d_ws.numel() * d_ws.element_size(), _stream(stream)))
    return plen.value


def prove_circuit_noalloc(c: Circuit, d_inputs, seed: int, d_outputs, d_proof, stream=None) -> int:
    """gkr_prove_circuit_noalloc (workspace in the library's static device
    array); returns the proof length."""
    plen = _sz(0)
    _check(lib().gkr_prove_circuit_noalloc(c.handle, _ptr(d_inputs), seed & (2**64 - 1), _ptr(d_outputs),
                                           _ptr(d_proof), d_proof.numel() * d_proof.element_size(),
                                           ctypes.byref(plen), _stream(stream)))
    return plen.value


def gl_device_elements(arr, device="cuda"):
    """Upload canonical Goldilocks elements (uint64) as a torch int64 tensor."""
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def gl_prove_circuit(c: Circuit, d_inputs, seed: int, d_outputs, d_proof, d_ws, stream=None) -> int:
    """gkr_gl_prove_circuit on caller tensors (int64 views of the elements)."""
    plen = _sz(0)
    _check(lib().gkr_gl_prove_circuit(c.handle, _ptr(d_inputs), seed & (2**64 - 1), _ptr(d_outputs),
                                      _ptr(d_proof), d_proof.numel() * d_proof.element_size(), ctypes.byref(plen),
                                      _ptr(d_ws), d_ws.numel() * d_ws.element_size(), _stream(stream)))
    return plen.value


def gl_verify(c: Circuit, inputs, outputs, seed: int, proof: bytes) -> int:
    """gkr_gl_verify on host buffers (uint64 elements)."""
    a = np.ascontiguousarray(inputs, dtype=np.uint64)
    b = np.ascontiguousarray(outputs, dtype=np.uint64)
    pb = np.frombuffer(bytes(proof), dtype=np.uint8)
    return _check(lib().gkr_gl_verify(c.handle, a.ctypes.data, b.ctypes.data, seed & (2**64 - 1),
                                      pb.ctypes.data if pb.size else None, pb.size))


class GlProver:
    """Device buffers of one Goldilocks proof at a time for one circuit."""

    def __init__(self, c: Circuit, device="cuda"):
        import torch
        self.c = c
        self.ws = alloc_bytes(c.workspace_bytes, device)
        self.proof = alloc_bytes(c.proof_bytes, device)
        self.outputs = torch.empty(1 << c.s(0), dtype=torch.int64, device=device)

    def prove(self, d_inputs, seed: int, stream=None) -> int:
        return gl_prove_circuit(self.c, d_inputs, seed, self.outputs, self.proof, self.ws, stream)

    def proof_bytes(self) -> bytes:
        return bytes(self.proof[: self.c.proof_bytes].cpu().numpy().tobytes())

    def host_outputs(self) -> np.ndarray:
        return self.outputs.cpu().numpy().view(np.uint64)


def transcript_init(c: Circuit, seed: int, d_inputs, d_outputs, d_state, d_ws, stream=None):
    _check(lib().gkr_transcript_init(c.handle, seed & (2**64 - 1), _ptr(d_inputs), _ptr(d_outputs), _ptr(d_state),
                                     _ptr(d_ws), d_ws.numel() * d_ws.element_size(), _stream(stream)))


def output_claim(c: Circuit, d_outputs, d_state, d_g, d_claim, d_ws, stream=None):
    _check(lib().gkr_output_claim(c.handle, _ptr(d_outputs), _ptr(d_state), _ptr(d_g), _ptr(d_claim), _ptr(d_ws),
                                  d_ws.numel() * d_ws.element_size(), _stream(stream)))


def prove_layer(c: Circuit, layer: int, d_next, d_u, d_v, d_claim_u, d_claim_v, d_state, d_rx, d_ry, d_vx,
                d_vy, d_layer_proof, d_ws, stream=None):
    _check(lib().gkr_prove_layer(c.handle, layer, _ptr(d_next), _ptr(d_u), _ptr(d_v), _ptr(d_claim_u),
                                 _ptr(d_claim_v), _ptr(d_state), _ptr(d_rx), _ptr(d_ry), _ptr(d_vx), _ptr(d_vy),
                                 _ptr(d_layer_proof), _ptr(d_ws), d_ws.numel() * d_ws.element_size(),
                                 _stream(stream)))


def verify(c: Circuit, inputs, outputs, seed: int, proof: bytes) -> int:
    """gkr_verify on host buffers: 1 accept, 0 reject (raises on malformed input)."""
    a, b = _elements(inputs), _elements(outputs)
    pb = np.frombuffer(bytes(proof), dtype=np.uint8)
    return _check(lib().gkr_verify(c.handle, a.ctypes.data, b.ctypes.data, seed & (2**64 - 1),
                                   pb.ctypes.data if pb.size else None, pb.size))


class Prover:
    """Owns the device buffers of one plain proof at a time for one circuit."""

    def __init__(self, c: Circuit, device="cuda"):
        import torch
        self.c = c
        self.device = device
        self.ws = alloc_bytes(c.workspace_bytes, device)
        self.proof = alloc_bytes(c.proof_bytes, device)
        self.outputs = torch.empty((1 << c.s(0), 8), dtype=torch.int32, device=device)

    def prove(self, d_inputs, seed: int, stream=None) -> int:
        return prove_circuit(self.c, d_inputs, seed, self.outputs, self.proof, self.ws, stream)

    def proof_bytes(self) -> bytes:
        return bytes(self.proof[: self.c.proof_bytes].cpu().numpy().tobytes())


# ------------------------------------------------------------ committed inputs

DEFAULT_QUERIES = 64


def committed_sizes(c: Circuit, queries: int = DEFAULT_QUERIES):
    """(workspace bytes, proof bytes) of a committed-input proof."""
    ws, pb = _sz(0), _sz(0)
    _check(lib().gkr_committed_sizes(c.handle, queries, ctypes.byref(ws), ctypes.byref(pb)))
    return ws.value, pb.value


def prove_circuit_committed(c: Circuit, d_inputs, seed: int, queries: int, d_outputs, d_proof, d_ws,
                            stream=None) -> None:
    """gkr_prove_circuit_committed on caller tensors."""
    _check(lib().gkr_prove_circuit_committed(c.handle, _ptr(d_inputs), seed & (2**64 - 1), queries,
                                             _ptr(d_outputs), _ptr(d_proof),
                                             d_proof.numel() * d_proof.element_size(), _ptr(d_ws),
                                             d_ws.numel() * d_ws.element_size(), _stream(stream)))


def verify_committed(c: Circuit, outputs, seed: int, proof: bytes, queries: int = DEFAULT_QUERIES) -> int:
    """gkr_verify_committed on host buffers (the outputs only): 1 accept, 0 reject."""
    b = _elements(outputs)
    pb = np.frombuffer(bytes(proof), dtype=np.uint8)
    return _check(lib().gkr_verify_committed(c.handle, b.ctypes.data, seed & (2**64 - 1), queries,
                                             pb.ctypes.data if pb.size else None, pb.size))


def vpd_workspace_bytes(log_n: int) -> int:
    n = _sz(0)
    _check(lib().gkr_vpd_workspace_bytes(log_n, ctypes.byref(n)))
    return n.value


def vpd_commit(log_n: int, d_values, d_root, d_ws, stream=None) -> None:
    """gkr_vpd_commit: the 32-byte root of the commitment to 2^log_n values."""
    _check(lib().gkr_vpd_commit(log_n, _ptr(d_values), _ptr(d_root), _ptr(d_ws),
                                d_ws.numel() * d_ws.element_size(), _stream(stream)))


class CommittedProver:
    """Device buffers of one committed-input proof at a time for one circuit."""

    def __init__(self, c: Circuit, queries: int = DEFAULT_QUERIES, device="cuda"):
        import torch
        self.c = c
        self.queries = queries
        ws, self.nbytes = committed_sizes(c, queries)
        self.ws = alloc_bytes(ws, device)
        self.proof = alloc_bytes(self.nbytes, device)
        self.outputs = torch.empty((1 << c.s(0), 8), dtype=torch.int32, device=device)

    def prove(self, d_inputs, seed: int, stream=None) -> None:
        prove_circuit_committed(self.c, d_inputs, seed, self.queries, self.outputs, self.proof, self.ws, stream)

    def proof_bytes(self) -> bytes:
        return bytes(self.proof[: self.nbytes].cpu().numpy().tobytes())


# ------------------------------------------------------------ batched proving

class Job(ctypes.Structure):
    _fields_ = [("circuit", _vp), ("d_inputs", _vp), ("seed", _u64), ("d_outputs", _vp), ("d_proof", _vp),
                ("proof_cap", _sz), ("d_ws", _vp), ("ws_bytes", _sz)]


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        L.gkr_plan_create.argtypes = [ctypes.POINTER(Job), ctypes.POINTER(_vp)]
        L.gkr_plan_create.restype = _i32
        L.gkr_plan_destroy.argtypes = [_vp]
        L.gkr_plan_destroy.restype = None
        L.gkr_plan_reset.argtypes = [_vp, _vp]
        L.gkr_plan_reset.restype = _i32
        L.gkr_run_batch.argtypes = [ctypes.POINTER(_vp), _u32, _vp, _u32, _u32, _u32, _vp]
        L.gkr_run_batch.restype = _i32
        L.gkr_plan_progress.argtypes = [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32)]
        L.gkr_plan_progress.restype = _i32
        L.gkr_prove_batch.argtypes = [ctypes.POINTER(Job), _u32, _vp]
        L.gkr_prove_batch.restype = _i32
        L.gkr_set_tuning.argtypes = [_u32, _u32, _u32]
        L.gkr_set_tuning.restype = _i32
        L.gkr_get_tuning.argtypes = [ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32)]
        L.gkr_set_contraction.argtypes = [_u32]
        L.gkr_set_contraction.restype = _i32
        L.gkr_get_tuning.restype = _i32
        L._batch_ready = True
    return L


def make_job(c: Circuit, d_inputs, seed: int, d_outputs, d_proof, d_ws) -> Job:
    return Job(c.handle.value, _ptr(d_inputs), seed & (2**64 - 1), _ptr(d_outputs), _ptr(d_proof),
               d_proof.numel() * d_proof.element_size(), _ptr(d_ws), d_ws.numel() * d_ws.element_size())


class Plan:
    """A job's proof program recorded in device memory (gkr_plan_create)."""

    def __init__(self, job: Job):
        self.job = job
        h = _vp()
        _check(_batch_lib().gkr_plan_create(ctypes.byref(job), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def reset(self, stream=None):
        _check(_batch_lib().gkr_plan_reset(self._h, _stream(stream)))

    def progress(self) -> Tuple[int, int]:
        d, t = _u32(0), _u32(0)
        _check(_batch_lib().gkr_plan_progress(self._h, ctypes.byref(d), ctypes.byref(t)))
        return d.value, t.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _batch_lib().gkr_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(plans: Sequence[Plan], d_ctl, workgroups: int = -1, step_budget: int = 0,
              stop_on_finish: bool = False, stream=None):
    """gkr_run_batch; workgroups=-1 uses the autotuned count (0 = fill the device)."""
    if workgroups < 0:
        workgroups = tuned_batch_workgroups()
    arr = (_vp * len(plans))(*[p.handle.value for p in plans])
    _check(_batch_lib().gkr_run_batch(arr, len(plans), _ptr(d_ctl), workgroups, step_budget,
                                      1 if stop_on_finish else 0, _stream(stream)))


def prove_batch(jobs: Sequence[Job], stream=None):
    arr = (Job * len(jobs))(*jobs)
    _check(_batch_lib().gkr_prove_batch(arr, len(jobs), _stream(stream)))


def set_tuning(tail_log: int, max_round_blocks: int, pairs_per_thread: int = 1):
    _check(_batch_lib().gkr_set_tuning(tail_log, max_round_blocks, pairs_per_thread))


def set_contraction(matrix_cores: bool):
    """Phase-2 copy contraction of plain proofs: on the int8 matrix cores where
    a layer qualifies (True, the default) or always the scalar pass."""
    _check(_batch_lib().gkr_set_contraction(1 if matrix_cores else 0))


UBENCH_KINDS = {0: "v_mad_u64_u32", 1: "v_mad_u64_u32 + v_addc (field multiply-accumulate)",
                2: "v_add_u32", 3: "v_mul_lo_u32 / v_mul_hi_u32", 4: "Montgomery field product",
                5: "HBM stream of a folding round (bytes/s)"}


def ubench(kind: int, iters: int = 2048) -> Tuple[float, float]:
    """gkr_ubench: (operations per second over the device, launch ms)."""
    rate, ms = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().gkr_ubench(kind, iters, ctypes.byref(rate), ctypes.byref(ms)))
    return rate.value, ms.value


def get_tuning() -> Tuple[int, int, int]:
    a, b, c = _u32(0), _u32(0), _u32(0)
    _check(_batch_lib().gkr_get_tuning(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value
