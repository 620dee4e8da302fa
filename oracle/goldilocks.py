"""The GKR prover and verifier over the Goldilocks field (TEST INFRASTRUCTURE ONLY).

Section 4.1 (choice of the finite field) names two candidate fields: BN254
and Goldilocks, p = 2^64 - 2^32 + 1, which makes the prover several times
faster but does not support pairings. This module is the oracle of the
Goldilocks variant of the layered data-parallel prover: the same protocol as
oracle/prover.py and oracle/verifier.py (GKR layer relation, Libra's two-phase
product sumcheck, claims combined with squeezed alpha, beta, bits bound from
the most significant, copies in the low bits), with elements and transcript
rules of this field:

  elements       canonical integers in [0, p), serialised as 8 bytes little-endian
  init           st = SHA256("SISU-GKR-GL-v1" || LE64(seed))
  absorb(t, m)   st = SHA256(st || t || m), t a four-byte tag
  accept         v = LE64(st[0:8]); while v >= p: st = SHA256(st || "GKRC"), recompute;
                 the challenge is v
  squeeze        st = SHA256(st || "GKRC"), then accept
  round(e0, e2)  st = C(st, LE64(e0) || LE64(e2) || 47 zero bytes || 0x01), then accept
                 (C the SHA-256 compression function; e1 = claim - e0 is not hashed)
  statement      absorb("GKRD", circuit digest (the layered circuit's)),
                 absorb("GKRD", tree digest of the inputs), absorb("GKRD", of the outputs)
  values         vx, vy absorbed with "GKRV"

The field arithmetic is Python integer arithmetic mod p; eq tables, folds and
multilinear extensions are written out here for this modulus. Parity status:
pinned (tests/test_oracle_goldilocks.py): field laws and p's structure,
transcript steps against hashlib and the FIPS compression function,
brute-force hypercube sums of every round polynomial on tiny circuits,
g_j(0) + g_j(1) = claim, verifier acceptance and tamper rejection.
"""
import dataclasses
import hashlib
import struct
from typing import List, Optional, Sequence

from .circuit import MUL, Circuit
from .transcript import TAG_CHALLENGE, TAG_DIGEST, TAG_VALUE, circuit_digest, compress, tree_digest

P = (1 << 64) - (1 << 32) + 1
ELEMENT_BYTES = 8
HALF = (P + 1) // 2
DOMAIN = b"SISU-GKR-GL-v1"


def to_bytes(a: int) -> bytes:
    if not 0 <= a < P:
        raise ValueError("element not canonical")
    return a.to_bytes(8, "little")


def from_bytes(b: bytes) -> int:
    if len(b) != 8:
        raise ValueError("element must be 8 bytes")
    v = int.from_bytes(b, "little")
    if v >= P:
        raise ValueError("element not canonical")
    return v


def encode_all(vals) -> bytes:
    return b"".join(to_bytes(v) for v in vals)


def vector_digest(values: Sequence[int]) -> bytes:
    return tree_digest(encode_all(values))


# ---------------------------------------------------------------- multilinear extensions

def eq_table(r: Sequence[int]) -> List[int]:
    """[eq(r, bits(b)) for b < 2^len(r)], variable 1 the most significant bit."""
    table = [1]
    for rk in r:
        nk = (1 - rk) % P
        table = [v for t in table for v in (t * nk % P, t * rk % P)]
    return table


def fold(table: Sequence[int], r: int) -> List[int]:
    h = len(table) // 2
    return [(a + r * (b - a)) % P for a, b in zip(table[:h], table[h:])]


def mle(table: Sequence[int], r: Sequence[int]) -> int:
    if len(table) != 1 << len(r):
        raise ValueError("table size does not match the point")
    x = list(table)
    for rj in r:
        x = fold(x, rj)
    return x[0]


def mle_by_eq(table: Sequence[int], r: Sequence[int]) -> int:
    return sum(v * e for v, e in zip(table, eq_table(r))) % P


# ---------------------------------------------------------------- transcript

class Transcript:
    def __init__(self, seed: int):
        self.state = hashlib.sha256(DOMAIN + struct.pack("<Q", seed & (2**64 - 1))).digest()

    def absorb(self, tag: bytes, data: bytes) -> None:
        self.state = hashlib.sha256(self.state + tag + data).digest()

    def absorb_elements(self, tag: bytes, values: Sequence[int]) -> None:
        self.absorb(tag, encode_all(values))

    def accept(self) -> int:
        v = int.from_bytes(self.state[:8], "little")
        while v >= P:
            self.state = hashlib.sha256(self.state + TAG_CHALLENGE).digest()
            v = int.from_bytes(self.state[:8], "little")
        return v

    def squeeze(self) -> int:
        self.state = hashlib.sha256(self.state + TAG_CHALLENGE).digest()
        return self.accept()

    def round_challenge(self, e0: int, e2: int) -> int:
        blk = to_bytes(e0) + to_bytes(e2) + bytes(47) + b"\x01"
        self.state = compress(self.state, blk)
        return self.accept()


# ---------------------------------------------------------------- evaluation

def evaluate(circuit: Circuit, inputs: Sequence[int]) -> List[List[int]]:
    """All layer values mod p (the layer relation of the GKR section)."""
    if len(inputs) != 1 << circuit.s(circuit.depth):
        raise ValueError("wrong input count")
    layers = [None] * (circuit.depth + 1)
    layers[circuit.depth] = list(inputs)
    for i in range(circuit.depth - 1, -1, -1):
        nxt = layers[i + 1]
        layers[i] = [(nxt[x] * nxt[y]) % P if t == MUL else (nxt[x] + nxt[y]) % P
                     for x, y, t in circuit.flat_gates(i)]
    return layers


# ---------------------------------------------------------------- prover

@dataclasses.dataclass
class LayerTrace:
    alpha: int
    beta: int
    claim: int
    messages1: List[List[int]]
    rx: List[int]
    vx: int
    messages2: List[List[int]]
    ry: List[int]
    vy: int

    def proof_bytes(self) -> bytes:
        out = [encode_all(m) for m in self.messages1] + [to_bytes(self.vx)]
        out += [encode_all(m) for m in self.messages2] + [to_bytes(self.vy)]
        return b"".join(out)


@dataclasses.dataclass
class ProofTrace:
    outputs: List[int]
    g: List[int]
    claim0: int
    layers: List[LayerTrace]

    def proof_bytes(self) -> bytes:
        return b"".join(l.proof_bytes() for l in self.layers)


def proof_length(circuit: Circuit) -> int:
    return sum((6 * circuit.s(i + 1) + 2) * ELEMENT_BYTES for i in range(circuit.depth))


def combined_eq(u, v, alpha: int, beta: int) -> List[int]:
    eu = eq_table(u)
    if v is None:
        return [alpha * a % P for a in eu]
    return [(alpha * a + beta * b) % P for a, b in zip(eu, eq_table(v))]


def sumcheck_product(W: List[int], X: List[int], Y: List[int], tr: Transcript):
    """Sumcheck of sum_b W[b] X[b] + Y[b] (degree-2 rounds sent at t = 0, 1, 2)."""
    messages, challenges = [], []
    while len(W) > 1:
        h = len(W) // 2
        e = []
        for t in (0, 1, 2):
            acc = 0
            for b in range(h):
                wt = W[b] + t * (W[b + h] - W[b])
                xt = X[b] + t * (X[b + h] - X[b])
                yt = Y[b] + t * (Y[b + h] - Y[b])
                acc += wt * xt + yt
            e.append(acc % P)
        r = tr.round_challenge(e[0], e[2])
        messages.append(e)
        challenges.append(r)
        W, X, Y = fold(W, r), fold(X, r), fold(Y, r)
    return messages, challenges, W[0]


def prove_layer(circuit: Circuit, i: int, W, u, v, alpha: int, beta: int, claim: int, tr: Transcript) -> LayerTrace:
    s1 = circuit.s(i + 1)
    gates = circuit.flat_gates(i)
    T = combined_eq(u, v, alpha, beta)
    G, H = [0] * (1 << s1), [0] * (1 << s1)
    for z, (x, y, t) in enumerate(gates):
        if t == MUL:
            G[x] += T[z] * W[y]
        else:
            G[x] += T[z]
            H[x] += T[z] * W[y]
    msgs1, rx, vx = sumcheck_product(list(W), [a % P for a in G], [a % P for a in H], tr)
    tr.absorb_elements(TAG_VALUE, [vx])
    E = eq_table(rx)
    M, A = [0] * (1 << s1), [0] * (1 << s1)
    for z, (x, y, t) in enumerate(gates):
        if t == MUL:
            M[y] += T[z] * E[x]
        else:
            A[y] += T[z] * E[x]
    F = [(vx * m + a) % P for m, a in zip(M, A)]
    K = [vx * a % P for a in A]
    msgs2, ry, vy = sumcheck_product(list(W), F, K, tr)
    tr.absorb_elements(TAG_VALUE, [vy])
    return LayerTrace(alpha, beta, claim, msgs1, rx, vx, msgs2, ry, vy)


def bind_statement(circuit: Circuit, inputs, outputs, seed: int) -> Transcript:
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, circuit_digest(circuit.depth, circuit.n, circuit.sigma, circuit.wiring))
    tr.absorb(TAG_DIGEST, vector_digest(inputs))
    tr.absorb(TAG_DIGEST, vector_digest(outputs))
    return tr


def prove(circuit: Circuit, inputs: Sequence[int], seed: int) -> ProofTrace:
    layers = evaluate(circuit, inputs)
    d = circuit.depth
    tr = bind_statement(circuit, layers[d], layers[0], seed)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    claim0 = mle(layers[0], g)
    traces = []
    u, v, vu, vv = g, None, claim0, 0
    for i in range(d):
        alpha, beta = (1, 0) if i == 0 else (tr.squeeze(), tr.squeeze())
        claim = (alpha * vu + beta * vv) % P
        lt = prove_layer(circuit, i, layers[i + 1], u, v, alpha, beta, claim, tr)
        traces.append(lt)
        u, v, vu, vv = lt.rx, lt.ry, lt.vx, lt.vy
    return ProofTrace(list(layers[0]), g, claim0, traces)


# ---------------------------------------------------------------- verifier

class MalformedProof(ValueError):
    pass


def interpolate(e: Sequence[int], r: int) -> int:
    e0, e1, e2 = e
    return (e0 * ((r - 1) * (r - 2) % P * HALF) - e1 * r * (r - 2) + e2 * (r * (r - 1) % P * HALF)) % P


def predicates(circuit: Circuit, i: int, u, v, alpha, beta, rx, ry):
    T = combined_eq(u, v, alpha, beta)
    ex, ey = eq_table(rx), eq_table(ry)
    add_v = mul_v = 0
    for z, (x, y, t) in enumerate(circuit.flat_gates(i)):
        term = T[z] * ex[x] % P * ey[y]
        if t == MUL:
            mul_v += term
        else:
            add_v += term
    return add_v % P, mul_v % P


def verify(circuit: Circuit, inputs: Sequence[int], outputs: Sequence[int], seed: int, proof: bytes) -> bool:
    d = circuit.depth
    if len(inputs) != 1 << circuit.s(d) or len(outputs) != 1 << circuit.s(0):
        raise ValueError("input or output vector has the wrong size")
    if any(not 0 <= a < P for a in list(inputs) + list(outputs)):
        raise ValueError("input or output element not canonical")
    if len(proof) != proof_length(circuit):
        raise MalformedProof("proof length %d, expected %d" % (len(proof), proof_length(circuit)))
    pos = 0

    def element():
        nonlocal pos
        try:
            val = from_bytes(proof[pos:pos + 8])
        except ValueError as exc:
            raise MalformedProof(str(exc)) from exc
        pos += 8
        return val

    tr = bind_statement(circuit, inputs, outputs, seed)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    accept = True
    u: List[int] = g
    v: Optional[List[int]] = None
    vu, vv = mle(list(outputs), g), 0
    for i in range(d):
        alpha, beta = (1, 0) if i == 0 else (tr.squeeze(), tr.squeeze())
        claim = (alpha * vu + beta * vv) % P
        s1 = circuit.s(i + 1)
        rs = [[], []]
        vals = [0, 0]
        for ph in range(2):
            for _ in range(s1):
                e = [element(), element(), element()]
                if (e[0] + e[1]) % P != claim:
                    accept = False
                r = tr.round_challenge(e[0], e[2])
                rs[ph].append(r)
                claim = interpolate(e, r)
            vals[ph] = element()
            tr.absorb_elements(TAG_VALUE, [vals[ph]])
        rx, ry = rs
        vx, vy = vals
        add_v, mul_v = predicates(circuit, i, u, v, alpha, beta, rx, ry)
        accept = accept and claim == (mul_v * vx % P * vy + add_v * (vx + vy)) % P
        u, v, vu, vv = rx, ry, vx, vy
    return accept and vu == mle(list(inputs), u) and vv == mle(list(inputs), v)
