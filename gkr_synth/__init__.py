"""Seeded synthetic workloads for the data-parallel GKR prover.

This module is the only code shared by the CPU oracle and the HIP path. It
draws circuits (wiring and gate types) and input vectors from counter-based
splitmix64 streams and carries none of the proving arithmetic: the only use of
the field modulus is the rejection test that makes sampled elements uniform
and canonical.

Workload shapes stand in for the paper's Ethereum validator circuits, which
are not available: layered fan-in-2 add/mul circuits made of 2^n identical
sub-circuit copies (the data-parallel structure of the GKR section and the
distributed sumcheck of Section 3.2.1), each gate wired uniformly at random
to the next layer of its own copy.

Index convention shared by every consumer: gate z of copy c in a layer with
sub-circuit width 2^sigma sits at global index g = z * 2^n + c (the copy in
the low bits), so a gate's inputs are x_z * 2^n + c and y_z * 2^n + c.

Elements are returned as numpy arrays of shape (count, 8) uint32 holding the
canonical value in little-endian 32-bit limbs.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# BN254 scalar field modulus (the element range for rejection sampling only).
MODULUS = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
_MOD_WORDS = [(MODULUS >> (64 * k)) & (2**64 - 1) for k in range(4)]

GATE_ADD = 0
GATE_MUL = 1

# splitmix64 (Steele, Lea, Flood: "Fast splittable pseudorandom number
# generators", OOPSLA 2014): state += GAMMA, output = mix64(state).
GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1

# Stream purposes.
PURPOSE_WIRE_X = 1
PURPOSE_WIRE_Y = 2
PURPOSE_GATE_TYPE = 3
PURPOSE_INPUT = 4
PURPOSE_JOB = 5
PURPOSE_ARRIVAL = 6
PURPOSE_NEST_COUNT = 7
PURPOSE_NEST_X = 8
PURPOSE_NEST_SRC = 9
PURPOSE_NEST_Y = 10
PURPOSE_NEST_TYPE = 11


def mix64(z: int) -> int:
    """splitmix64 output finaliser on a Python int (mod 2^64)."""
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, purpose: int, layer: int = 0) -> int:
    """Key of the stream for (seed, purpose, layer)."""
    return mix64(mix64(seed ^ 0x53495355474B5231) ^ ((purpose << 32) | (layer & 0xFFFFFFFF)))


def stream(key: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the splitmix64 stream whose state starts at `key`.

    Output i is mix64(key + (i + 1) * GAMMA), so any output can be computed alone.
    """
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        st = idx * np.uint64(GAMMA) + np.uint64(key)
        return _mix64_np(st)


def stream_at(key: int, i: int) -> int:
    return mix64(key + (i + 1) * GAMMA)


# ---------------------------------------------------------------- elements

def _less_than_modulus(w: Sequence[np.ndarray]) -> np.ndarray:
    """Lexicographic (w3, w2, w1, w0) < MODULUS, vectorised."""
    lt = np.zeros(w[0].shape, dtype=bool)
    eq = np.ones(w[0].shape, dtype=bool)
    for k in (3, 2, 1, 0):
        pk = np.uint64(_MOD_WORDS[k])
        lt |= eq & (w[k] < pk)
        eq &= w[k] == pk
    return lt


def field_elements(key: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform canonical field elements start..start+count-1 of the element stream `key`.

    Large ranges are split into blocks generated on a thread pool (each element
    depends only on its own index, so the split does not change the values).
    """
    block = 1 << 20
    if count <= 2 * block:
        return _field_elements_block(key, count, start)
    import concurrent.futures
    import os
    out = np.empty((count, 8), dtype=np.uint32)
    starts = list(range(0, count, block))
    workers = max(1, min(16, os.cpu_count() or 1))

    def fill(off):
        n = min(block, count - off)
        out[off:off + n] = _field_elements_block(key, n, start + off)

    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(fill, starts))
    return out


def _field_elements_block(key: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform canonical field elements start..start+count-1 of the element stream `key`.

    Element k draws its own sub-stream with state stream_at(key, k); attempt a
    takes that sub-stream's outputs 4a..4a+3 as little-endian 64-bit words,
    keeps the low 254 bits, and is accepted when the value is below the modulus
    (acceptance about 0.756 per attempt).
    """
    out = np.zeros((count, 4), dtype=np.uint64)
    if count == 0:
        return out.view(np.uint32).reshape(count, 8)
    sub = stream(key, count, start)
    pending = np.arange(count, dtype=np.int64)
    attempt = 0
    with np.errstate(over="ignore"):
        while pending.size:
            base = sub[pending]
            words = [
                _mix64_np(base + np.uint64(((4 * attempt + j + 1) * GAMMA) & _M64))
                for j in range(4)
            ]
            words[3] = words[3] & np.uint64((1 << 62) - 1)
            ok = _less_than_modulus(words)
            acc = pending[ok]
            for j in range(4):
                out[acc, j] = words[j][ok]
            pending = pending[~ok]
            attempt += 1
    return out.view(np.uint32).reshape(count, 8)


def elements_to_ints(arr: np.ndarray) -> List[int]:
    """(count, 8) uint32 limbs -> Python ints (format conversion only)."""
    a = np.ascontiguousarray(arr, dtype=np.uint32).view(np.uint64).reshape(-1, 4)
    return [int(r[0]) | (int(r[1]) << 64) | (int(r[2]) << 128) | (int(r[3]) << 192) for r in a]


def ints_to_elements(vals: Sequence[int]) -> np.ndarray:
    """Python ints in [0, 2^256) -> (count, 8) uint32 limbs (format conversion only)."""
    out = np.zeros((len(vals), 4), dtype=np.uint64)
    for i, v in enumerate(vals):
        for k in range(4):
            out[i, k] = (v >> (64 * k)) & _M64
    return out.view(np.uint32).reshape(len(vals), 8)


# ---------------------------------------------------------------- circuits

@dataclasses.dataclass(frozen=True)
class CircuitSpec:
    """Shape of a layered data-parallel circuit.

    depth            number of gate layers d (layer 0 is the output, layer d the input)
    log_copies       n: the circuit is 2^n copies of one sub-circuit
    log_sub_width    sigma_0..sigma_d: log2 of the sub-circuit width of each layer
    mu               fraction of MUL gates as (numerator, denominator)
    seed             workload seed
    """

    depth: int
    log_copies: int
    log_sub_width: Tuple[int, ...]
    mu: Tuple[int, int] = (1, 2)
    seed: int = 1

    def __post_init__(self):
        if len(self.log_sub_width) != self.depth + 1:
            raise ValueError("log_sub_width needs depth + 1 entries")

    def log_width(self, i: int) -> int:
        return self.log_sub_width[i] + self.log_copies

    @property
    def gate_layers(self) -> int:
        """Sum over gate layers of 2^{s_i}: the field-gate count of one proof."""
        return sum(1 << self.log_width(i) for i in range(self.depth))


@dataclasses.dataclass
class Wiring:
    """Sub-circuit wiring of one gate layer: arrays indexed by local gate z."""

    x: np.ndarray  # uint32, local index into the next layer
    y: np.ndarray  # uint32
    kind: np.ndarray  # uint32, GATE_ADD or GATE_MUL


def make_wiring(spec: CircuitSpec) -> List[Wiring]:
    """Uniform random wiring of each layer's sub-circuit (x = y allowed)."""
    num, den = spec.mu
    threshold = (num << 64) // den
    out = []
    for i in range(spec.depth):
        width = 1 << spec.log_sub_width[i]
        mask = np.uint64((1 << spec.log_sub_width[i + 1]) - 1)
        x = (stream(stream_key(spec.seed, PURPOSE_WIRE_X, i), width) & mask).astype(np.uint32)
        y = (stream(stream_key(spec.seed, PURPOSE_WIRE_Y, i), width) & mask).astype(np.uint32)
        t = stream(stream_key(spec.seed, PURPOSE_GATE_TYPE, i), width)
        if threshold >= 1 << 64:
            kind = np.full(width, GATE_MUL, dtype=np.uint32)
        else:
            kind = np.where(t < np.uint64(threshold), GATE_MUL, GATE_ADD).astype(np.uint32)
        out.append(Wiring(x, y, kind))
    return out


def make_inputs(spec: CircuitSpec, start: int = 0, count: Optional[int] = None) -> np.ndarray:
    """Input layer V_d (or a slice of it) as canonical (count, 8) uint32 limbs."""
    total = 1 << spec.log_width(spec.depth)
    if count is None:
        count = total - start
    if start < 0 or start + count > total:
        raise ValueError("input slice out of range")
    return field_elements(stream_key(spec.seed, PURPOSE_INPUT, 0), count, start)


def copy_slice(spec: CircuitSpec, log_copies: int) -> CircuitSpec:
    """The same sub-circuit with fewer copies (a bounded sample of a workload)."""
    return dataclasses.replace(spec, log_copies=log_copies)


# ---------------------------------------------------------------- workloads

def plain_c1() -> CircuitSpec:
    """One layered circuit: depth 4, 2^10 gates per layer, half MUL gates."""
    return CircuitSpec(depth=4, log_copies=0, log_sub_width=(10,) * 5, mu=(1, 2), seed=1)


def data_parallel_c2() -> CircuitSpec:
    """2^8 copies of a depth-16 sub-circuit with 2^12 gates per layer (2^20 per layer)."""
    return CircuitSpec(depth=16, log_copies=8, log_sub_width=(12,) * 17, mu=(1, 2), seed=2)


def worker_share_c3() -> CircuitSpec:
    """2^12 copies of a depth-24 sub-circuit with 2^14 gates per layer, 30 % MUL gates."""
    return CircuitSpec(depth=24, log_copies=12, log_sub_width=(14,) * 25, mu=(3, 10), seed=3)


def _job_shape(seed: int, s_lo: int, s_hi: int, d_lo: int, d_hi: int) -> CircuitSpec:
    w = stream(stream_key(seed, PURPOSE_JOB, 0), 3)
    s = s_lo + int(w[0] % np.uint64(s_hi - s_lo + 1))
    d = d_lo + int(w[1] % np.uint64(d_hi - d_lo + 1))
    n_hi = min(10, s - 4)
    n = 4 + int(w[2] % np.uint64(n_hi - 4 + 1))
    return CircuitSpec(depth=d, log_copies=n, log_sub_width=(s - n,) * (d + 1), mu=(1, 2), seed=seed)


def batch_jobs_c4(count: int = 64, first_seed: int = 1000) -> List[CircuitSpec]:
    """Uneven batch: log2 width uniform in [10, 18], depth uniform in [8, 32], 2^4..2^10 copies."""
    return [_job_shape(first_seed + k, 10, 18, 8, 32) for k in range(count)]


def serving_jobs_c5(count: int = 256, trace_seed: int = 2000) -> List[CircuitSpec]:
    """Serving mix: log2 width uniform in [12, 22], depth uniform in [8, 24]."""
    return [_job_shape(trace_seed * 1000 + k, 12, 22, 8, 24) for k in range(count)]


def poisson_gaps(count: int, rate: float, trace_seed: int = 2000) -> np.ndarray:
    """Seeded exponential inter-arrival gaps (seconds) of a Poisson stream of the given rate."""
    w = stream(stream_key(trace_seed, PURPOSE_ARRIVAL, 0), count)
    u = (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))  # [0, 1)
    return -np.log1p(-u) / rate


# ---------------------------------------------------------------- general circuits

@dataclasses.dataclass(frozen=True)
class GeneralSpec:
    """Shape of a general (non-layered) data-parallel circuit with accumulation gates.

    Gate z of gate layer i holds 1..max_fanin nested fan-in-2 gates (uniform);
    each reads its left input x from layer i+1 and its right input y from layer
    i+1 or, with probability `cross`, from one of the layers i+2 .. i+reach
    (uniform; capped at the input layer); MUL with probability mu.

    depth, log_copies, log_sub_width, mu, seed  as in CircuitSpec
    max_fanin   nested gates per gate: uniform in [1, max_fanin]
    reach       right inputs come from layers i+1 .. min(depth, i + reach)
    cross       probability (numerator, denominator) of a right input beyond layer i+1
    """

    depth: int
    log_copies: int
    log_sub_width: Tuple[int, ...]
    max_fanin: int = 2
    reach: int = 3
    cross: Tuple[int, int] = (1, 4)
    mu: Tuple[int, int] = (1, 2)
    seed: int = 1

    def __post_init__(self):
        if len(self.log_sub_width) != self.depth + 1:
            raise ValueError("log_sub_width needs depth + 1 entries")
        if self.max_fanin < 1 or self.reach < 1:
            raise ValueError("max_fanin and reach must be at least 1")

    def log_width(self, i: int) -> int:
        return self.log_sub_width[i] + self.log_copies

    @property
    def gate_layers(self) -> int:
        """Sum over gate layers of 2^{s_i} (gates, not nested gates)."""
        return sum(1 << self.log_width(i) for i in range(self.depth))


@dataclasses.dataclass
class NestedWiring:
    """The nested gates of one gate layer's sub-circuit, grouped by output gate z
    (ascending): output z, left input x (layer i+1), right-input layer src, right
    input y (layer src), type."""

    z: np.ndarray    # uint32
    x: np.ndarray    # uint32
    src: np.ndarray  # uint32
    y: np.ndarray    # uint32
    kind: np.ndarray  # uint32, GATE_ADD or GATE_MUL


def make_general_wiring(spec: GeneralSpec) -> List[NestedWiring]:
    """Seeded nested-gate lists of every gate layer (see GeneralSpec)."""
    num, den = spec.mu
    mul_threshold = (num << 64) // den
    cnum, cden = spec.cross
    cross_threshold = (cnum << 32) // cden
    d = spec.depth
    out = []
    for i in range(d):
        width = 1 << spec.log_sub_width[i]
        cnt = (stream(stream_key(spec.seed, PURPOSE_NEST_COUNT, i), width) % np.uint64(spec.max_fanin)
               + np.uint64(1)).astype(np.int64)
        total = int(cnt.sum())
        z = np.repeat(np.arange(width, dtype=np.uint32), cnt)
        x = (stream(stream_key(spec.seed, PURPOSE_NEST_X, i), total)
             & np.uint64((1 << spec.log_sub_width[i + 1]) - 1)).astype(np.uint32)
        hi = min(d, i + spec.reach)
        w = stream(stream_key(spec.seed, PURPOSE_NEST_SRC, i), total)
        src = np.full(total, i + 1, dtype=np.uint32)
        if hi > i + 1:
            far = (w >> np.uint64(32)) < np.uint64(cross_threshold)
            pick = (i + 2 + (w & np.uint64(0xFFFFFFFF)) % np.uint64(hi - i - 1)).astype(np.uint32)
            src = np.where(far, pick, src).astype(np.uint32)
        ymask = np.array([(1 << spec.log_sub_width[j]) - 1 if j <= d else 0 for j in range(d + 1)],
                         dtype=np.uint64)
        y = (stream(stream_key(spec.seed, PURPOSE_NEST_Y, i), total) & ymask[src]).astype(np.uint32)
        t = stream(stream_key(spec.seed, PURPOSE_NEST_TYPE, i), total)
        if mul_threshold >= 1 << 64:
            kind = np.full(total, GATE_MUL, dtype=np.uint32)
        else:
            kind = np.where(t < np.uint64(mul_threshold), GATE_MUL, GATE_ADD).astype(np.uint32)
        out.append(NestedWiring(z, x, src, y, kind))
    return out


def make_general_inputs(spec: GeneralSpec, start: int = 0, count: Optional[int] = None) -> np.ndarray:
    """Input layer V_d of a general circuit (same element stream as make_inputs)."""
    total = 1 << spec.log_width(spec.depth)
    if count is None:
        count = total - start
    if start < 0 or start + count > total:
        raise ValueError("input slice out of range")
    return field_elements(stream_key(spec.seed, PURPOSE_INPUT, 0), count, start)


def general_small() -> GeneralSpec:
    """A small general circuit for parity: 2^4 copies x depth 6, 2^8 gates per layer,
    up to 4 nested gates per gate, right inputs up to 3 layers back."""
    return GeneralSpec(depth=6, log_copies=4, log_sub_width=(8,) * 7, max_fanin=4, reach=3, cross=(1, 3),
                       mu=(1, 2), seed=40)


def general_data_parallel() -> GeneralSpec:
    """General-circuit workload: 2^8 copies x depth 8, 2^12 gates per layer, up to 4 nested
    gates per gate (accumulation gates), a quarter of the right inputs from 2..4 layers back."""
    return GeneralSpec(depth=8, log_copies=8, log_sub_width=(12,) * 9, max_fanin=4, reach=4, cross=(1, 4),
                       mu=(1, 2), seed=41)


# ---------------------------------------------------------------- Goldilocks elements

GOLDILOCKS = (1 << 64) - (1 << 32) + 1  # the modulus (element range for rejection sampling only)


def goldilocks_elements(key: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform canonical Goldilocks elements start..start+count-1 of the element
    stream `key`: element k takes output a of its own sub-stream (state
    stream_at(key, k)) for attempt a = 0, 1, ... and accepts the first value
    below the modulus (acceptance 1 - 2^-32 per attempt). uint64 array."""
    out = np.zeros(count, dtype=np.uint64)
    if count == 0:
        return out
    sub = stream(key, count, start)
    pending = np.arange(count, dtype=np.int64)
    attempt = 0
    with np.errstate(over="ignore"):
        while pending.size:
            w = _mix64_np(sub[pending] + np.uint64(((attempt + 1) * GAMMA) & _M64))
            ok = w < np.uint64(GOLDILOCKS)
            out[pending[ok]] = w[ok]
            pending = pending[~ok]
            attempt += 1
    return out


def make_goldilocks_inputs(spec: CircuitSpec, start: int = 0, count: Optional[int] = None) -> np.ndarray:
    """Input layer V_d of a layered circuit over the Goldilocks field (uint64)."""
    total = 1 << spec.log_width(spec.depth)
    if count is None:
        count = total - start
    if start < 0 or start + count > total:
        raise ValueError("input slice out of range")
    return goldilocks_elements(stream_key(spec.seed, PURPOSE_INPUT, 0), count, start)
