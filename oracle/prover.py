"""GKR prover with the two-phase linear-time sumcheck (GKR and Libra sections).

For gate layer i with W = V_{i+1} (2^{s'} values, s' = s_{i+1}) the prover
reduces a claim about V_i~ to claims about W~ at two random points.

Claim combination. Layer 0 has one claim V_0~(g). Every later layer receives two
points (u, v) = (r_x, r_y) with values (V_i~(u), V_i~(v)); it draws alpha, beta
from the transcript and proves alpha V_i~(u) + beta V_i~(v). With
T[z] = alpha eq(u, z) + beta eq(v, z) (T = eq(g, .) on layer 0):

  sum_z T[z] V_i[z] = sum_x W[x] G[x] + H[x]                 (phase 1, over x)
      G[x] = sum_{MUL z, x_z = x} T[z] W[y_z] + sum_{ADD z, x_z = x} T[z]
      H[x] = sum_{ADD z, x_z = x} T[z] W[y_z]

After phase 1 binds x to r_x with vx = W~(r_x), with E = eq(r_x, .):

  vx G~(r_x) + H~(r_x) = sum_y W[y] F[y] + K[y]               (phase 2, over y)
      M[y] = sum_{MUL z, y_z = y} T[z] E[x_z],  A[y] = sum_{ADD z, y_z = y} T[z] E[x_z]
      F = vx M + A,  K = vx A

Each phase is the Libra product sumcheck over bookkeeping tables: in round j
the prover sends the degree-2 round polynomial through its values at t = 0, 1, 2,
e_t = sum_{b < M/2} W_t[b] X_t[b] + Y_t[b] with X_t[b] = X[b] + t (X[b+M/2] - X[b]),
then halves every table by the challenge r_j (the table-update step).

Proof bytes of a layer: phase-1 messages (s' x 96 B), vx, phase-2 messages, vy.
"""
import dataclasses
from typing import List, Optional, Sequence

from . import mle
from .circuit import MUL, Circuit, evaluate
from .field import P, encode_all, to_bytes
from .transcript import TAG_DIGEST, TAG_VALUE, Transcript, circuit_digest, vector_digest


@dataclasses.dataclass
class LayerTrace:
    alpha: int
    beta: int
    claim: int                      # alpha V_i~(u) + beta V_i~(v), the phase-1 start claim
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


def combined_eq(u: Sequence[int], v: Optional[Sequence[int]], alpha: int, beta: int) -> List[int]:
    """T[z] = alpha eq(u, z) + beta eq(v, z); v is None on the output layer."""
    eu = mle.eq_table(u)
    if v is None:
        return [alpha * a % P for a in eu]
    ev = mle.eq_table(v)
    return [(alpha * a + beta * b) % P for a, b in zip(eu, ev)]


def sumcheck_product(W: List[int], X: List[int], Y: List[int], tr: Transcript):
    """Sumcheck of sum_b W[b] X[b] + Y[b]; returns (messages, challenges, final W value)."""
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
        W, X, Y = mle.fold(W, r), mle.fold(X, r), mle.fold(Y, r)
    return messages, challenges, W[0]


def prove_layer(circuit: Circuit, i: int, W: Sequence[int], u: Sequence[int],
                v: Optional[Sequence[int]], alpha: int, beta: int, claim: int,
                tr: Transcript) -> LayerTrace:
    s1 = circuit.s(i + 1)
    if len(W) != 1 << s1:
        raise ValueError("W has the wrong size")
    gates = circuit.flat_gates(i)
    T = combined_eq(u, v, alpha, beta)

    # Phase 1 bookkeeping tables.
    G = [0] * (1 << s1)
    H = [0] * (1 << s1)
    for z, (x, y, t) in enumerate(gates):
        if t == MUL:
            G[x] += T[z] * W[y]
        else:
            G[x] += T[z]
            H[x] += T[z] * W[y]
    G = [a % P for a in G]
    H = [a % P for a in H]
    msgs1, rx, vx = sumcheck_product(list(W), G, H, tr)
    tr.absorb_elements(TAG_VALUE, [vx])

    # Phase 2 bookkeeping tables.
    E = mle.eq_table(rx)
    M = [0] * (1 << s1)
    A = [0] * (1 << s1)
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


def bind_statement(circuit: Circuit, inputs: Sequence[int], outputs: Sequence[int], seed: int) -> Transcript:
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, circuit_digest(circuit.depth, circuit.n, circuit.sigma, circuit.wiring))
    tr.absorb(TAG_DIGEST, vector_digest(inputs))
    tr.absorb(TAG_DIGEST, vector_digest(outputs))
    return tr


def prove_from_layers(circuit: Circuit, layers: List[List[int]], seed: int) -> ProofTrace:
    d = circuit.depth
    tr = bind_statement(circuit, layers[d], layers[0], seed)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    claim0 = mle.evaluate(layers[0], g)
    traces = []
    u, v, vu, vv = g, None, claim0, 0
    for i in range(d):
        if i == 0:
            alpha, beta = 1, 0
        else:
            alpha, beta = tr.squeeze(), tr.squeeze()
        claim = (alpha * vu + beta * vv) % P
        lt = prove_layer(circuit, i, layers[i + 1], u, v, alpha, beta, claim, tr)
        traces.append(lt)
        u, v, vu, vv = lt.rx, lt.ry, lt.vx, lt.vy
    return ProofTrace(list(layers[0]), g, claim0, traces)


def prove(circuit: Circuit, inputs: Sequence[int], seed: int) -> ProofTrace:
    """Outputs and proof of the statement 'outputs = circuit(inputs)'."""
    return prove_from_layers(circuit, evaluate(circuit, inputs), seed)


def proof_length(circuit: Circuit) -> int:
    return sum((6 * circuit.s(i + 1) + 2) * 32 for i in range(circuit.depth))
