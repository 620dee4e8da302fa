"""General circuits with accumulation gates: evaluation, GKR prover and verifier
(TEST INFRASTRUCTURE ONLY).

Section 2.7 (general arithmetic circuit): a gate of layer i may read a gate of
any later layer j, as long as one of its inputs is in layer i+1; for a pair of
layers (i, j) only the gates of layer j that layer i actually reads are
indexed, so the sumcheck over j's values runs over those gates only.
Section 3.4.3 (accumulation gate): a gate holds a list of nested fan-in-2
gates, possibly of different types and reading different layers, and its
value is the sum of the nested gates' values; the layer relation of the GKR
section is unchanged, an output gate simply has several (x, y) terms.

Model used here (both the oracle and the HIP path; see the design notes for
the readings of the paper):
  - gate layer i holds nested gates (z, x, j, y, type): output gate z of layer
    i, left input x in layer i+1, right input y in layer j (i < j <= d);
    V_i[z] = sum over z's nested gates of V_{i+1}[x] + V_j[y] (ADD) or
    V_{i+1}[x] V_j[y] (MUL); data-parallel copies as in the layered circuit
    (gate z of copy c is z * 2^n + c and reads x * 2^n + c, y * 2^n + c);
  - used gates: U_{i,j} = the distinct y's layer i reads from layer j, sorted.
    Layer i's right-input vector R_i concatenates the used gates of its source
    layers j_0 < j_1 < ... as blocks: R_i[((b 2^tau_i + k) 2^n) + c] =
    V_{j_b}[U_{i,j_b}[k] 2^n + c], zero where k >= |U_{i,j_b}| or b >= the
    number of sources; 2^beta_i blocks of 2^tau_i entries (beta_i, tau_i the
    bit counts of the source count and of the largest used set);
    rho_i = beta_i + tau_i + n. A nested gate's right index is
    y' = b(j) 2^tau_i + position of y in U_{i,j}.
  - the layer relation becomes V_i(g) = sum over nested gates of
    add (V_{i+1}(x) + R_i(y')) + mult V_{i+1}(x) R_i(y'), proved with the
    two-phase sumcheck: phase 1 over x (s_{i+1} variables, tables W = V_{i+1},
    G, H), phase 2 over y' (rho_i variables, tables R_i, F, K);
  - claims: after phase 2 the prover sends, for every source block b, the
    value v_b = MLE of block b at the local and copy parts of r_y; the
    verifier checks R_i~(r_y) = sum_b eq(r_y[:beta], b) v_b. Each v_b is a
    linear claim on V_{j_b}: sum_{k, c} eq(r_loc, k) eq(r_cp, c)
    V_{j_b}[U[k] 2^n + c]. Layer i+1 also receives the eq claim V_{i+1}~(r_x)
    = vx from phase 1. A layer's claims are combined with one squeezed
    coefficient each (layer 0 has the single claim V_0~(g), coefficient 1),
    in the order they were produced. The input layer's claims are checked by
    the verifier directly from the inputs.
  - proof of layer i: s_{i+1} phase-1 messages, vx, rho_i phase-2 messages,
    vy, then one value per source block (absorbed one by one with "GKRV").

Parity status: pinned (tests/test_oracle_general.py): forward evaluation by
hand and against the layered oracle, brute-force hypercube sums of every
round polynomial from the multilinear predicates (no bookkeeping tables),
the concatenation identity, every claim against its definition, verifier
acceptance and tamper rejection.
"""
import dataclasses
import struct
from typing import Dict, List, Optional, Sequence, Tuple

from . import mle
from .circuit import ADD, MUL
from .field import P, encode_all, from_bytes, to_bytes
from .prover import sumcheck_product
from .transcript import TAG_DIGEST, TAG_VALUE, Transcript, sha256, vector_digest
from .verifier import MalformedProof, _check_phase

GENERAL_DOMAIN = b"GKR-GENERAL-v1"


def bit_count(count: int) -> int:
    """Number of index bits for `count` entries (0 for one entry)."""
    b = 0
    while (1 << b) < count:
        b += 1
    return b


class GeneralCircuit:
    def __init__(self, depth: int, log_copies: int, log_sub_width: Sequence[int], layers):
        """layers[i] = nested gates (z, x, src, y, type) of gate layer i."""
        if depth < 1:
            raise ValueError("a circuit needs at least one gate layer")
        if len(log_sub_width) != depth + 1 or len(layers) != depth:
            raise ValueError("shape mismatch")
        self.depth = depth
        self.n = log_copies
        self.sigma = [int(s) for s in log_sub_width]
        self.records: List[List[Tuple[int, int, int, int, int]]] = []
        for i, recs in enumerate(layers):
            recs = [tuple(int(v) for v in r) for r in recs]
            if not recs:
                raise ValueError("gate layer %d has no nested gates" % i)
            for z, x, j, y, t in recs:
                if not (0 <= z < 1 << self.sigma[i] and 0 <= x < 1 << self.sigma[i + 1]):
                    raise ValueError("layer %d: output or left input out of range" % i)
                if not (i < j <= depth and 0 <= y < 1 << self.sigma[j]):
                    raise ValueError("layer %d: right input out of range" % i)
                if t not in (ADD, MUL):
                    raise ValueError("unknown gate type")
            self.records.append(recs)
        # used gates of each source layer and the block layout of R_i
        self.sources: List[List[int]] = []
        self.used: List[Dict[int, List[int]]] = []
        self.pos: List[Dict[int, Dict[int, int]]] = []
        self.beta, self.tau = [], []
        for recs in self.records:
            srcs = sorted({j for _, _, j, _, _ in recs})
            used = {j: sorted({y for _, _, jj, y, _ in recs if jj == j}) for j in srcs}
            self.sources.append(srcs)
            self.used.append(used)
            self.pos.append({j: {y: k for k, y in enumerate(u)} for j, u in used.items()})
            self.beta.append(bit_count(len(srcs)))
            self.tau.append(max(bit_count(len(u)) for u in used.values()))

    @classmethod
    def from_synth(cls, spec, wiring) -> "GeneralCircuit":
        layers = [list(zip(w.z.tolist(), w.x.tolist(), w.src.tolist(), w.y.tolist(), w.kind.tolist()))
                  for w in wiring]
        return cls(spec.depth, spec.log_copies, spec.log_sub_width, layers)

    def s(self, i: int) -> int:
        return self.sigma[i] + self.n

    def rho(self, i: int) -> int:
        """Variables of layer i's phase 2 (log2 of R_i's size)."""
        return self.beta[i] + self.tau[i] + self.n

    def right_index(self, i: int, j: int, y: int) -> int:
        """Local index y' of (layer j, gate y) in R_i."""
        b = self.sources[i].index(j)
        return (b << self.tau[i]) | self.pos[i][j][y]

    def flat_records(self, i: int) -> List[Tuple[int, int, int, int]]:
        """Global nested gates of layer i: (g, x, y', type) with copy bits appended."""
        n = self.n
        out = []
        for z, x, j, y, t in self.records[i]:
            yl = self.right_index(i, j, y)
            for c in range(1 << n):
                out.append(((z << n) | c, (x << n) | c, (yl << n) | c, t))
        return out

    def gate_layers(self) -> int:
        return sum(1 << self.s(i) for i in range(self.depth))

    def nested_gates(self) -> int:
        return sum(len(r) for r in self.records) << self.n


def digest(c: GeneralCircuit) -> bytes:
    """SHA256("GKR-GENERAL-v1" || LE32 d || LE32 n || LE32 sigma_0..sigma_d || for each
    gate layer: LE32 count || each nested gate: LE32 z, x, src, y || u8 type)."""
    parts = [GENERAL_DOMAIN, struct.pack("<II", c.depth, c.n)]
    parts += [struct.pack("<I", s) for s in c.sigma]
    for recs in c.records:
        parts.append(struct.pack("<I", len(recs)))
        parts += [struct.pack("<IIIIB", z, x, j, y, t) for z, x, j, y, t in recs]
    return sha256(b"".join(parts))


# ---------------------------------------------------------------- evaluation

def evaluate(c: GeneralCircuit, inputs: Sequence[int]) -> List[List[int]]:
    """All layer values, from the definition: each gate sums its nested gates,
    each nested gate reading V_{i+1}[x] and V_j[y] directly."""
    if len(inputs) != 1 << c.s(c.depth):
        raise ValueError("wrong input count")
    n = c.n
    layers: List[Optional[List[int]]] = [None] * (c.depth + 1)
    layers[c.depth] = list(inputs)
    for i in range(c.depth - 1, -1, -1):
        out = [0] * (1 << c.s(i))
        nxt = layers[i + 1]
        for z, x, j, y, t in c.records[i]:
            src = layers[j]
            for cp in range(1 << n):
                a, b = nxt[(x << n) | cp], src[(y << n) | cp]
                out[(z << n) | cp] += a * b if t == MUL else a + b
        layers[i] = [v % P for v in out]
    return layers


def right_vector(c: GeneralCircuit, i: int, layers) -> List[int]:
    """R_i: the used gates of each source layer as consecutive blocks (zero padded)."""
    n = c.n
    R = [0] * (1 << c.rho(i))
    for b, j in enumerate(c.sources[i]):
        for k, y in enumerate(c.used[i][j]):
            for cp in range(1 << n):
                R[(((b << c.tau[i]) | k) << n) | cp] = layers[j][(y << n) | cp]
    return R


# ---------------------------------------------------------------- claims

@dataclasses.dataclass
class Claim:
    """A claim about layer `layer`: sum_g weight[g] V[g] = value. kind "eq": the
    weight is eq(point, .); kind "subset": the weight of gate used[k] * 2^n + c is
    eq(point[:tau], k) eq(point[tau:], c) (zero elsewhere), tau = len(point) - n."""
    layer: int
    kind: str
    point: List[int]
    value: int
    used: Optional[List[int]] = None


def claim_weights(c: GeneralCircuit, cl: Claim) -> List[int]:
    if cl.kind == "eq":
        return mle.eq_table(cl.point)
    n = c.n
    tau = len(cl.point) - n
    el, ec = mle.eq_table(cl.point[:tau]), mle.eq_table(cl.point[tau:])
    w = [0] * (1 << c.s(cl.layer))
    for k, z in enumerate(cl.used):
        for cp in range(1 << n):
            w[(z << n) | cp] = el[k] * ec[cp] % P
    return w


def combined_weights(c: GeneralCircuit, claims: Sequence[Claim], coefs: Sequence[int]) -> List[int]:
    """T = sum_k coef_k weight_k."""
    T = [0] * (1 << c.s(claims[0].layer))
    for cl, a in zip(claims, coefs):
        for g, w in enumerate(claim_weights(c, cl)):
            T[g] += a * w
    return [t % P for t in T]


# ---------------------------------------------------------------- prover

@dataclasses.dataclass
class GeneralLayerTrace:
    coefs: List[int]
    claim: int
    messages1: List[List[int]]
    rx: List[int]
    vx: int
    messages2: List[List[int]]
    ry: List[int]
    vy: int
    block_values: List[int]

    def proof_bytes(self) -> bytes:
        out = [encode_all(m) for m in self.messages1] + [to_bytes(self.vx)]
        out += [encode_all(m) for m in self.messages2] + [to_bytes(self.vy)]
        out += [to_bytes(v) for v in self.block_values]
        return b"".join(out)


@dataclasses.dataclass
class GeneralProofTrace:
    outputs: List[int]
    g: List[int]
    claim0: int
    layers: List[GeneralLayerTrace]
    input_claims: List[Claim]

    def proof_bytes(self) -> bytes:
        return b"".join(l.proof_bytes() for l in self.layers)


def proof_length(c: GeneralCircuit) -> int:
    return sum((3 * c.s(i + 1) + 3 * c.rho(i) + 2 + len(c.sources[i])) * 32 for i in range(c.depth))


def bind_statement(c: GeneralCircuit, inputs, outputs, seed: int) -> Transcript:
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, digest(c))
    tr.absorb(TAG_DIGEST, vector_digest(inputs))
    tr.absorb(TAG_DIGEST, vector_digest(outputs))
    return tr


def prove_layer(c: GeneralCircuit, i: int, layers, claims: Sequence[Claim], tr: Transcript):
    """One gate layer: returns the layer trace and the claims it hands to later layers."""
    n = c.n
    coefs = [1] if i == 0 else [tr.squeeze() for _ in claims]
    T = combined_weights(c, claims, coefs)
    claim = sum(a * cl.value for a, cl in zip(coefs, claims)) % P
    W = layers[i + 1]
    R = right_vector(c, i, layers)
    recs = c.flat_records(i)
    # phase 1 over x: sum_x W[x] G[x] + H[x]
    G = [0] * len(W)
    H = [0] * len(W)
    for g, x, y, t in recs:
        if t == MUL:
            G[x] += T[g] * R[y]
        else:
            G[x] += T[g]
            H[x] += T[g] * R[y]
    msgs1, rx, vx = sumcheck_product(list(W), [v % P for v in G], [v % P for v in H], tr)
    tr.absorb_elements(TAG_VALUE, [vx])
    # phase 2 over y': sum_y' R[y'] F[y'] + K[y']
    E = mle.eq_table(rx)
    M = [0] * len(R)
    A = [0] * len(R)
    for g, x, y, t in recs:
        if t == MUL:
            M[y] += T[g] * E[x]
        else:
            A[y] += T[g] * E[x]
    F = [(vx * m + a) % P for m, a in zip(M, A)]
    K = [vx * a % P for a in A]
    msgs2, ry, vy = sumcheck_product(list(R), F, K, tr)
    tr.absorb_elements(TAG_VALUE, [vy])
    # one value per source block: block b of R_i at the local and copy parts of r_y
    beta, tau = c.beta[i], c.tau[i]
    local = ry[beta:]
    size = 1 << (tau + n)
    vals, out_claims = [], [Claim(i + 1, "eq", list(rx), vx)]
    for b, j in enumerate(c.sources[i]):
        v = mle.evaluate(R[b * size:(b + 1) * size], local)
        tr.absorb_elements(TAG_VALUE, [v])
        vals.append(v)
        out_claims.append(Claim(j, "subset", list(local), v, list(c.used[i][j])))
    lt = GeneralLayerTrace(coefs, claim, msgs1, rx, vx, msgs2, ry, vy, vals)
    return lt, out_claims


def prove_from_layers(c: GeneralCircuit, layers, seed: int) -> GeneralProofTrace:
    d = c.depth
    tr = bind_statement(c, layers[d], layers[0], seed)
    g = [tr.squeeze() for _ in range(c.s(0))]
    claim0 = mle.evaluate(layers[0], g)
    pending: List[List[Claim]] = [[] for _ in range(d + 1)]
    pending[0].append(Claim(0, "eq", g, claim0))
    traces = []
    for i in range(d):
        lt, out = prove_layer(c, i, layers, pending[i], tr)
        traces.append(lt)
        for cl in out:
            pending[cl.layer].append(cl)
    return GeneralProofTrace(list(layers[0]), g, claim0, traces, pending[d])


def prove(c: GeneralCircuit, inputs, seed: int) -> GeneralProofTrace:
    return prove_from_layers(c, evaluate(c, inputs), seed)


# ---------------------------------------------------------------- verifier

def predicates(c: GeneralCircuit, i: int, T, rx, ry) -> Tuple[int, int]:
    """(add~, mult~) at (r_x, r_y) weighted by T, from the flattened nested gates."""
    ex, ey = mle.eq_table(rx), mle.eq_table(ry)
    add_v = mul_v = 0
    for g, x, y, t in c.flat_records(i):
        term = T[g] * ex[x] % P * ey[y]
        if t == MUL:
            mul_v += term
        else:
            add_v += term
    return add_v % P, mul_v % P


class _Reader:
    def __init__(self, data: bytes):
        self.data, self.pos = data, 0

    def element(self) -> int:
        if self.pos + 32 > len(self.data):
            raise MalformedProof("proof too short")
        try:
            v = from_bytes(self.data[self.pos:self.pos + 32])
        except ValueError as exc:
            raise MalformedProof(str(exc)) from exc
        self.pos += 32
        return v


def verify(c: GeneralCircuit, inputs: Sequence[int], outputs: Sequence[int], seed: int, proof: bytes) -> bool:
    d, n = c.depth, c.n
    if len(inputs) != 1 << c.s(d) or len(outputs) != 1 << c.s(0):
        raise ValueError("input or output vector has the wrong size")
    if any(not 0 <= a < P for a in inputs) or any(not 0 <= a < P for a in outputs):
        raise ValueError("input or output element not canonical")
    if len(proof) != proof_length(c):
        raise MalformedProof("proof length %d, expected %d" % (len(proof), proof_length(c)))
    rd = _Reader(proof)
    tr = bind_statement(c, inputs, outputs, seed)
    g = [tr.squeeze() for _ in range(c.s(0))]
    pending: List[List[Claim]] = [[] for _ in range(d + 1)]
    pending[0].append(Claim(0, "eq", g, mle.evaluate(list(outputs), g)))
    accept = True
    for i in range(d):
        claims = pending[i]
        coefs = [1] if i == 0 else [tr.squeeze() for _ in claims]
        claim = sum(a * cl.value for a, cl in zip(coefs, claims)) % P
        ok1, claim, rx = _check_phase(rd, c.s(i + 1), claim, tr)
        vx = rd.element()
        tr.absorb_elements(TAG_VALUE, [vx])
        ok2, claim, ry = _check_phase(rd, c.rho(i), claim, tr)
        vy = rd.element()
        tr.absorb_elements(TAG_VALUE, [vy])
        vals = []
        for _ in c.sources[i]:
            v = rd.element()
            tr.absorb_elements(TAG_VALUE, [v])
            vals.append(v)
        beta = c.beta[i]
        eb = mle.eq_table(ry[:beta])
        ok3 = vy == sum(e * v for e, v in zip(eb, vals)) % P
        T = combined_weights(c, claims, coefs)
        add_v, mul_v = predicates(c, i, T, rx, ry)
        ok4 = claim == (mul_v * vx % P * vy + add_v * (vx + vy)) % P
        accept = accept and ok1 and ok2 and ok3 and ok4
        pending[i + 1].append(Claim(i + 1, "eq", list(rx), vx))
        for v, j in zip(vals, c.sources[i]):
            pending[j].append(Claim(j, "subset", list(ry[beta:]), v, list(c.used[i][j])))
    # the input layer: every claim straight from the inputs
    for cl in pending[d]:
        w = claim_weights(c, cl)
        accept = accept and cl.value == sum(a * b for a, b in zip(w, inputs)) % P
    return accept
