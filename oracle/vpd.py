"""Commitment to the input layer and its opening at the two final points (TEST INFRASTRUCTURE ONLY).

Section 2.4 (Virgo protocol): instead of reading the input layer V_D, the
verifier has the prover commit to V_D~ before the GKR protocol runs; when the
last layer leaves two claims V_D~(r_x) = v_x and V_D~(r_y) = v_y, the prover
opens the commitment at those two points. Virgo's commitment (a verifiable
polynomial delegation) is transparent and built on the univariate sumcheck;
the paper gives no more detail. This module is the oracle of this project's
reading of it:

  polynomial   the N = 2^s inputs are the coefficients of f(X) = sum_b V[b] X^b.
  claim        with w[b] = eq(r1, b) + lam eq(r2, b) (variable 1 = the most
               significant bit of b, as everywhere in this project) the two claims
               become c = c1 + lam c2 = sum_b V[b] w[b].
  tensor       sum_b eq(r, b) Y^b = prod_j ((1 - r_j) + r_j Y^(2^(s-j))) =: Q_r(Y),
               Q = Q_r1 + lam Q_r2, evaluated in O(s) operations at any Y.
  sumcheck     H = the order-N subgroup, q(X) = sum_b w[b] X^((N - b) mod N), so
               q(x) = Q(1/x) on H and q(x) = x^N Q(1/x) + (1 - x^N) Q(0) anywhere.
               sum_{x in H} f(x) q(x) = N c. The prover splits p = f q as
               p = g + (X^N - 1) h with deg g < N, so g(0) = c, and sends
               g' = (g - c) / X and h. Identity checked at a point x:
               f(x) q(x) = c + x g'(x) + (x^N - 1) h(x).
  low degree   FRI on R = a0 f + a1 h + a2 g' + a3 X g' (degree < N) over the coset
               L = 5 <w_M>, M = 4N (N <= 2^26: p - 1 has 2-adicity 28), folded s
               times down to a constant: R'(x^2) = (R(x) + R(-x)) / 2 + beta (R(x) - R(-x)) / (2x).
  storage      a table over a coset of size m is stored in bit-reversed order
               (position t holds the value at gamma w_m^bitrev(t)), so the pair
               (x, -x) sits at positions (2u, 2u + 1) and folding maps positions
               (2u, 2u + 1) of layer i to position u of layer i + 1.
  Merkle       leaf u of a table = its positions 2u, 2u + 1 (f and the FRI layers:
               one 64-byte block) or h, g' at both (128 bytes); elements enter
               as their Montgomery forms (e 2^256 mod p, 32 bytes little-endian,
               as in the transcript). A leaf digest is the SHA-256 compression
               function chained from the initial hash value over the 64-byte
               blocks (no padding: every leaf of a tree has the same length);
               a node is one compression of left || right from the initial value.
  transcript   the GKR statement absorbs root(f) in place of the input digest.
               After the last layer: lam = squeeze; absorb("GKRM", root(h, g'));
               a0..a3 = squeeze; for i < s: beta_i = squeeze, then (i + 1 < s)
               absorb("GKRM", root of layer i + 1); absorb("GKRV", final constant);
               query j: u_j = squeeze mod (M / 2), a leaf of the first layer.
  proof        root(f) || GKR layers || root(h, g') || roots 1..s-1 || final ||
               per query: f leaf (2 elements) and path, (h, g') leaf (4 elements)
               and path, then for layers i = 1..s-1 leaf u_j >> i (2 elements)
               and path; paths bottom-up; elements canonical little-endian.

Parity status: pinned (tests/test_oracle_vpd.py): the NTT against Horner
evaluation, the roots of unity and the coset against their definitions, the
tensor polynomial against the eq table, the univariate sumcheck identity and
the split of p, FRI folds against the coefficient fold, Merkle trees against
hashlib-padded SHA-256 and hand-built trees, acceptance of honest proofs and
rejection of tampered ones, of a wrong claim and of a high-degree codeword.
"""
import dataclasses
import struct
from typing import List, Optional, Sequence

from . import mle
from .circuit import Circuit, evaluate
from .field import P, to_bytes
from .prover import LayerTrace, prove_layer
from .transcript import SHA256_IV, TAG_DIGEST, TAG_VALUE, Transcript, circuit_digest, compress, vector_digest
from .verifier import MalformedProof, _check_phase, predicates_factored

TAG_COMMIT = b"GKRM"
TWO_ADICITY = 28
GENERATOR = 5                                   # a non-residue: 5^((p-1)/2^28) has order exactly 2^28
ROOT_OF_UNITY = pow(GENERATOR, (P - 1) >> TWO_ADICITY, P)
SHIFT = GENERATOR                               # the coset shift: 5^(2^28) != 1, so 5 <w_M> misses <w_M>
LOG_BLOWUP = 2
MAX_LOG_N = TWO_ADICITY - LOG_BLOWUP
DEFAULT_QUERIES = 64
_R = (1 << 256) % P


IV = struct.pack(">8I", *SHA256_IV)   # FIPS 180-4 Section 5.3.3, the initial hash value


# ---------------------------------------------------------------- domains and polynomials

def root_of_unity(m: int) -> int:
    """A generator of the order-m subgroup (m a power of two, m <= 2^28)."""
    if m < 1 or m & (m - 1) or m > 1 << TWO_ADICITY:
        raise ValueError("subgroup order must be a power of two up to 2^28")
    return pow(ROOT_OF_UNITY, (1 << TWO_ADICITY) // m, P)


def bitrev(i: int, k: int) -> int:
    return int(format(i, "0%db" % k)[::-1], 2) if k else 0


def ntt(a: Sequence[int], omega: int) -> List[int]:
    """[A(omega^k) for k < n], A(X) = sum_j a[j] X^j, n = len(a) a power of two
    (radix-2 decimation in time, plain recursion)."""
    n = len(a)
    if n == 1:
        return [a[0] % P]
    even = ntt(a[0::2], omega * omega % P)
    odd = ntt(a[1::2], omega * omega % P)
    out = [0] * n
    w = 1
    for k in range(n // 2):
        t = w * odd[k] % P
        out[k] = (even[k] + t) % P
        out[k + n // 2] = (even[k] - t) % P
        w = w * omega % P
    return out


def intt(vals: Sequence[int], omega: int) -> List[int]:
    n = len(vals)
    inv_n = pow(n, -1, P)
    return [v * inv_n % P for v in ntt(vals, pow(omega, -1, P))]


def poly_eval(coeffs: Sequence[int], x: int) -> int:
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % P
    return acc


def poly_mul(a: Sequence[int], b: Sequence[int]) -> List[int]:
    """Product coefficients (length len(a) + len(b) - 1) through NTTs of a
    power-of-two size at least that long."""
    size = len(a) + len(b) - 1
    n = 1
    while n < size:
        n *= 2
    w = root_of_unity(n)
    fa = ntt(list(a) + [0] * (n - len(a)), w)
    fb = ntt(list(b) + [0] * (n - len(b)), w)
    return intt([x * y % P for x, y in zip(fa, fb)], w)[:size]


def coset_values(coeffs: Sequence[int], m: int, shift: int) -> List[int]:
    """[F(shift w_m^k) for k < m] in natural order (deg F < m)."""
    if len(coeffs) > m:
        raise ValueError("more coefficients than domain points")
    scaled = [c * pow(shift, j, P) % P for j, c in enumerate(coeffs)] + [0] * (m - len(coeffs))
    return ntt(scaled, root_of_unity(m))


def to_bitrev(vals: Sequence[int]) -> List[int]:
    k = len(vals).bit_length() - 1
    return [vals[bitrev(t, k)] for t in range(len(vals))]


def point_of_position(t: int, m: int, shift: int) -> int:
    """The domain point stored at position t of a bit-reversed coset table."""
    return shift * pow(root_of_unity(m), bitrev(t, m.bit_length() - 1), P) % P


def tensor_eval(r: Sequence[int], y: int) -> int:
    """Q_r(y) = sum_b eq(r, bits(b)) y^b = prod_j ((1 - r_j) + r_j y^(2^(s-j)))."""
    s = len(r)
    acc = 1
    for j, rj in enumerate(r):
        acc = acc * ((1 - rj) + rj * pow(y, 1 << (s - 1 - j), P)) % P
    return acc


def q_at(r1: Sequence[int], r2: Sequence[int], lam: int, x: int) -> int:
    """q(x) for q(X) = sum_b w[b] X^((N - b) mod N), w = eq(r1, .) + lam eq(r2, .)."""
    n = 1 << len(r1)
    xn = pow(x, n, P)
    qinv = (tensor_eval(r1, pow(x, -1, P)) + lam * tensor_eval(r2, pow(x, -1, P))) % P
    q0 = (tensor_eval(r1, 0) + lam * tensor_eval(r2, 0)) % P
    return (xn * qinv + (1 - xn) * q0) % P


# ---------------------------------------------------------------- Merkle trees

def mont_bytes(a: int) -> bytes:
    return (a * _R % P).to_bytes(32, "little")


def chain(data: bytes) -> bytes:
    """The compression function chained from the initial value over 64-byte blocks."""
    if not data or len(data) % 64:
        raise ValueError("leaf data must be a whole number of 64-byte blocks")
    st = IV
    for i in range(0, len(data), 64):
        st = compress(st, data[i:i + 64])
    return st


class MerkleTree:
    """levels[0] = leaf digests, levels[-1] = [root]; the leaf count is a power of two."""

    def __init__(self, leaves: Sequence[bytes]):
        if not leaves or len(leaves) & (len(leaves) - 1):
            raise ValueError("leaf count must be a power of two")
        self.levels = [[chain(l) for l in leaves]]
        while len(self.levels[-1]) > 1:
            lv = self.levels[-1]
            self.levels.append([compress(IV, lv[2 * i] + lv[2 * i + 1]) for i in range(len(lv) // 2)])

    @property
    def root(self) -> bytes:
        return self.levels[-1][0]

    def path(self, u: int) -> List[bytes]:
        out = []
        for lv in self.levels[:-1]:
            out.append(lv[u ^ 1])
            u >>= 1
        return out


def root_from_path(leaf_digest: bytes, u: int, path: Sequence[bytes]) -> bytes:
    h = leaf_digest
    for sib in path:
        h = compress(IV, sib + h) if u & 1 else compress(IV, h + sib)
        u >>= 1
    return h


def pair_leaves(table: Sequence[int]) -> List[bytes]:
    return [mont_bytes(table[2 * u]) + mont_bytes(table[2 * u + 1]) for u in range(len(table) // 2)]


def quad_leaves(ta: Sequence[int], tb: Sequence[int]) -> List[bytes]:
    return [mont_bytes(ta[2 * u]) + mont_bytes(ta[2 * u + 1]) + mont_bytes(tb[2 * u]) + mont_bytes(tb[2 * u + 1])
            for u in range(len(ta) // 2)]


# ---------------------------------------------------------------- commitment

def domain_size(log_n: int) -> int:
    if not 0 <= log_n <= MAX_LOG_N:
        raise ValueError("the commitment supports 2^0 .. 2^%d inputs" % MAX_LOG_N)
    return 1 << (log_n + LOG_BLOWUP)


@dataclasses.dataclass
class Commitment:
    coeffs: List[int]
    table: List[int]          # f on L, bit-reversed positions
    tree: MerkleTree

    @property
    def root(self) -> bytes:
        return self.tree.root


def commit(values: Sequence[int]) -> Commitment:
    n = len(values)
    if n < 1 or n & (n - 1):
        raise ValueError("input count must be a power of two")
    m = domain_size(n.bit_length() - 1)
    table = to_bitrev(coset_values(list(values), m, SHIFT))
    return Commitment(list(values), table, MerkleTree(pair_leaves(table)))


def _fold_pair(pair: Sequence[int], beta: int, x: int) -> int:
    """R'(x^2) = (R(x) + R(-x)) / 2 + beta (R(x) - R(-x)) / (2x) from pair = (R(x), R(-x))."""
    a, b = pair
    half = (P + 1) // 2
    return ((a + b) * half + beta * (a - b) * half * pow(x, -1, P)) % P


def fold_table(table: Sequence[int], beta: int, shift: int) -> List[int]:
    """One FRI fold of a bit-reversed coset table: positions (2u, 2u + 1) hold
    R(x), R(-x); position u of the result holds R'(x^2)."""
    m = len(table)
    return [_fold_pair(table[2 * u:2 * u + 2], beta, point_of_position(2 * u, m, shift)) for u in range(m // 2)]


def split_product(f: Sequence[int], q: Sequence[int], c: int):
    """p = f q = g + (X^N - 1) h with deg g < N; returns (g', h) with g = c + X g'
    as coefficient lists of length N (the top entries are zero)."""
    n = len(f)
    p = poly_mul(f, q) + [0]
    p += [0] * (2 * n - len(p))
    g = [(p[k] + p[k + n]) % P for k in range(n)]
    h = [p[k + n] for k in range(n)]
    if g[0] != c % P:
        raise ValueError("the claimed value is not the sum over H / N")
    gp = g[1:] + [0]
    return gp, h


@dataclasses.dataclass
class QueryOpening:
    index: int
    f_leaf: List[int]
    f_path: List[bytes]
    hg_leaf: List[int]
    hg_path: List[bytes]
    layers: List[List[int]]
    layer_paths: List[List[bytes]]

    def proof_bytes(self) -> bytes:
        out = [b"".join(to_bytes(v) for v in self.f_leaf), b"".join(self.f_path),
               b"".join(to_bytes(v) for v in self.hg_leaf), b"".join(self.hg_path)]
        for vals, path in zip(self.layers, self.layer_paths):
            out.append(b"".join(to_bytes(v) for v in vals) + b"".join(path))
        return b"".join(out)


@dataclasses.dataclass
class Opening:
    lam: int
    root_hg: bytes
    coeffs_a: List[int]
    betas: List[int]
    roots: List[bytes]
    final: int
    queries: List[QueryOpening]

    def proof_bytes(self) -> bytes:
        out = [self.root_hg] + list(self.roots) + [to_bytes(self.final)]
        return b"".join(out) + b"".join(q.proof_bytes() for q in self.queries)


def opening_length(log_n: int, queries: int = DEFAULT_QUERIES) -> int:
    s = log_n
    depth0 = s + LOG_BLOWUP - 1
    per_query = (2 + depth0) + (4 + depth0) + sum(2 + depth0 - i for i in range(1, s))
    return 32 * (1 + max(s - 1, 0) + 1 + queries * per_query)


def open_at(com: Commitment, r1: Sequence[int], r2: Sequence[int], c1: int, c2: int, tr: Transcript,
            queries: int = DEFAULT_QUERIES, check_degree: bool = True) -> Opening:
    """Open f at r1 and r2 (claims c1, c2), continuing the transcript tr.
    check_degree=False lets the tests play a prover whose committed table is
    not of low degree (it sends the first entry of the last fold as the constant)."""
    n = len(com.coeffs)
    s = n.bit_length() - 1
    if len(r1) != s or len(r2) != s:
        raise ValueError("points must have log2(N) coordinates")
    m = domain_size(s)
    lam = tr.squeeze()
    c = (c1 + lam * c2) % P
    w = [(a + lam * b) % P for a, b in zip(mle.eq_table(r1), mle.eq_table(r2))]
    q = [w[(n - j) % n] for j in range(n)]
    gp, h = split_product(com.coeffs, q, c)
    h_tab = to_bitrev(coset_values(h, m, SHIFT))
    g_tab = to_bitrev(coset_values(gp, m, SHIFT))
    hg_tree = MerkleTree(quad_leaves(h_tab, g_tab))
    tr.absorb(TAG_COMMIT, hg_tree.root)
    a = [tr.squeeze() for _ in range(4)]
    R = []
    for t in range(m):
        x = point_of_position(t, m, SHIFT)
        R.append((a[0] * com.table[t] + a[1] * h_tab[t] + (a[2] + a[3] * x) * g_tab[t]) % P)
    layers, trees, betas, roots = [R], [], [], []
    shift = SHIFT
    for i in range(s):
        beta = tr.squeeze()
        betas.append(beta)
        nxt = fold_table(layers[-1], beta, shift)
        shift = shift * shift % P
        layers.append(nxt)
        if i + 1 < s:
            t = MerkleTree(pair_leaves(nxt))
            trees.append(t)
            roots.append(t.root)
            tr.absorb(TAG_COMMIT, t.root)
    final = layers[-1][0]
    if check_degree and any(v != final for v in layers[-1]):
        raise ValueError("the folded table is not constant: R has degree >= N")
    tr.absorb(TAG_VALUE, to_bytes(final))
    opened = []
    for _ in range(queries):
        u = tr.squeeze() % (m // 2)
        lv, lp = [], []
        for i in range(1, s):
            leaf = u >> i
            lv.append([layers[i][2 * leaf], layers[i][2 * leaf + 1]])
            lp.append(trees[i - 1].path(leaf))
        opened.append(QueryOpening(u, [com.table[2 * u], com.table[2 * u + 1]], com.tree.path(u),
                                   [h_tab[2 * u], h_tab[2 * u + 1], g_tab[2 * u], g_tab[2 * u + 1]],
                                   hg_tree.path(u), lv, lp))
    return Opening(lam, hg_tree.root, a, betas, roots, final, opened)


class _Reader:
    def __init__(self, data: bytes, pos: int = 0):
        self.data, self.pos = data, pos

    def raw(self, k: int) -> bytes:
        if self.pos + k > len(self.data):
            raise MalformedProof("proof too short")
        b = self.data[self.pos:self.pos + k]
        self.pos += k
        return b

    def element(self) -> int:
        v = int.from_bytes(self.raw(32), "little")
        if v >= P:
            raise MalformedProof("element not canonical")
        return v

    def digests(self, k: int) -> List[bytes]:
        return [self.raw(32) for _ in range(k)]


def verify_opening(root_f: bytes, log_n: int, r1: Sequence[int], r2: Sequence[int], c1: int, c2: int,
                   tr: Transcript, rd: _Reader, queries: int = DEFAULT_QUERIES) -> bool:
    """Check an opening read from rd against root_f, continuing the transcript tr."""
    s = log_n
    m = domain_size(s)
    n = 1 << s
    depth0 = s + LOG_BLOWUP - 1
    lam = tr.squeeze()
    c = (c1 + lam * c2) % P
    root_hg = rd.raw(32)
    tr.absorb(TAG_COMMIT, root_hg)
    a = [tr.squeeze() for _ in range(4)]
    betas, roots = [], []
    for i in range(s):
        betas.append(tr.squeeze())
        if i + 1 < s:
            roots.append(rd.raw(32))
            tr.absorb(TAG_COMMIT, roots[-1])
    final = rd.element()
    tr.absorb(TAG_VALUE, to_bytes(final))
    ok = True
    for _ in range(queries):
        u = tr.squeeze() % (m // 2)
        fv = [rd.element(), rd.element()]
        fpath = rd.digests(depth0)
        hg = [rd.element() for _ in range(4)]
        hgpath = rd.digests(depth0)
        ok = ok and root_from_path(chain(mont_bytes(fv[0]) + mont_bytes(fv[1])), u, fpath) == root_f
        ok = ok and root_from_path(chain(b"".join(mont_bytes(v) for v in hg)), u, hgpath) == root_hg
        # positions 2u and 2u + 1 of the first layer hold the points x and -x
        x = point_of_position(2 * u, m, SHIFT)
        pair = []
        for xx, fx, hx, gx in ((x, fv[0], hg[0], hg[2]), ((P - x) % P, fv[1], hg[1], hg[3])):
            ok = ok and fx * q_at(r1, r2, lam, xx) % P == (c + xx * gx + (pow(xx, n, P) - 1) * hx) % P
            pair.append((a[0] * fx + a[1] * hx + (a[2] + a[3] * xx) * gx) % P)
        if s == 0:
            ok = ok and pair[0] == final and pair[1] == final
            continue
        cur = _fold_pair(pair, betas[0], x)
        pos, size, shift = u, m // 2, SHIFT * SHIFT % P       # cur sits at position pos of layer 1
        for i in range(1, s):
            pair = [rd.element(), rd.element()]
            leaf = pos >> 1
            path = rd.digests(depth0 - i)
            ok = ok and root_from_path(chain(mont_bytes(pair[0]) + mont_bytes(pair[1])), leaf, path) == roots[i - 1]
            ok = ok and pair[pos & 1] == cur
            cur = _fold_pair(pair, betas[i], point_of_position(2 * leaf, size, shift))
            pos, size, shift = leaf, size // 2, shift * shift % P
        ok = ok and cur == final
    return ok


# ---------------------------------------------------------------- GKR with a committed input layer

@dataclasses.dataclass
class CommittedProof:
    outputs: List[int]
    root: bytes
    layers: List[LayerTrace]
    opening: Opening

    def proof_bytes(self) -> bytes:
        return self.root + b"".join(l.proof_bytes() for l in self.layers) + self.opening.proof_bytes()


def bind_statement_committed(circuit: Circuit, root: bytes, outputs: Sequence[int], seed: int) -> Transcript:
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, circuit_digest(circuit.depth, circuit.n, circuit.sigma, circuit.wiring))
    tr.absorb(TAG_DIGEST, root)
    tr.absorb(TAG_DIGEST, vector_digest(outputs))
    return tr


def prove_committed(circuit: Circuit, inputs: Sequence[int], seed: int,
                    queries: int = DEFAULT_QUERIES) -> CommittedProof:
    """The GKR proof of outputs = circuit(inputs) whose verifier holds only the
    commitment to the inputs, followed by the opening at the last layer's points."""
    if circuit.depth < 1:
        raise ValueError("a committed proof needs at least one gate layer")
    layers = evaluate(circuit, inputs)
    d = circuit.depth
    com = commit(layers[d])
    tr = bind_statement_committed(circuit, com.root, layers[0], seed)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    u, v, vu, vv = g, None, mle.evaluate(layers[0], g), 0
    traces = []
    for i in range(d):
        alpha, beta = (1, 0) if i == 0 else (tr.squeeze(), tr.squeeze())
        claim = (alpha * vu + beta * vv) % P
        lt = prove_layer(circuit, i, layers[i + 1], u, v, alpha, beta, claim, tr)
        traces.append(lt)
        u, v, vu, vv = lt.rx, lt.ry, lt.vx, lt.vy
    opening = open_at(com, u, v, vu, vv, tr, queries)
    return CommittedProof(list(layers[0]), com.root, traces, opening)


def committed_proof_length(circuit: Circuit, queries: int = DEFAULT_QUERIES) -> int:
    gkr = sum((6 * circuit.s(i + 1) + 2) * 32 for i in range(circuit.depth))
    return 32 + gkr + opening_length(circuit.s(circuit.depth), queries)


def verify_committed(circuit: Circuit, outputs: Sequence[int], seed: int, proof: bytes,
                     queries: int = DEFAULT_QUERIES) -> bool:
    """True iff the proof convinces a verifier that holds the outputs but not the inputs."""
    d = circuit.depth
    if d < 1:
        raise ValueError("a committed proof needs at least one gate layer")
    if len(outputs) != 1 << circuit.s(0) or any(not 0 <= a < P for a in outputs):
        raise ValueError("output vector has the wrong size or a non-canonical element")
    if len(proof) != committed_proof_length(circuit, queries):
        raise MalformedProof("proof length %d, expected %d" % (len(proof), committed_proof_length(circuit, queries)))
    root = proof[:32]
    from .verifier import _Reader as GkrReader
    rd = GkrReader(proof[32:])
    tr = bind_statement_committed(circuit, root, outputs, seed)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    accept = True
    u: List[int] = g
    v: Optional[List[int]] = None
    vu, vv = mle.evaluate(list(outputs), g), 0
    for i in range(d):
        alpha, beta = (1, 0) if i == 0 else (tr.squeeze(), tr.squeeze())
        claim = (alpha * vu + beta * vv) % P
        s1 = circuit.s(i + 1)
        ok1, claim, rx = _check_phase(rd, s1, claim, tr)
        vx = rd.element()
        tr.absorb_elements(TAG_VALUE, [vx])
        ok2, claim, ry = _check_phase(rd, s1, claim, tr)
        vy = rd.element()
        tr.absorb_elements(TAG_VALUE, [vy])
        add_v, mul_v = predicates_factored(circuit, i, u, v, alpha, beta, rx, ry)
        accept = accept and ok1 and ok2 and (mul_v * vx % P * vy + add_v * (vx + vy)) % P == claim
        u, v, vu, vv = rx, ry, vx, vy
    vrd = _Reader(proof, 32 + rd.pos)
    return verify_opening(root, circuit.s(d), u, v, vu, vv, tr, vrd, queries) and accept
