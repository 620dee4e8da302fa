"""GKR verifier (GKR section; the round check of Section 3.2.1).

For every round the verifier checks g_j(0) + g_j(1) = current claim, then moves
the claim to g_j(r_j) (degree-2 Lagrange interpolation through t = 0, 1, 2).
After phase 2 of layer i the claim must equal

    mult~(r_x, r_y) vx vy + add~(r_x, r_y) (vx + vy),
    mult~(r_x, r_y) = sum_{MUL z} T[z] eq(r_x, x_z) eq(r_y, y_z)   (add~ likewise over ADD gates)

with T[z] = alpha eq(u, z) + beta eq(v, z). The next layer's claims are vx, vy
at (r_x, r_y); after the last layer the verifier evaluates the input MLE at both
points itself (the paper's Virgo variant would open a polynomial commitment
instead; here the verifier reads the inputs).

Two predicate evaluators are provided: `generic` sums over the flattened global
gate list (O(2^s)); `factored` uses the data-parallel structure, summing over the
sub-circuit gates once and closing the copy bits with the product
sum_c eq(a, c) eq(b, c) eq(d, c) = prod_k (a_k b_k d_k + (1-a_k)(1-b_k)(1-d_k)),
which is O(2^sigma + n) per layer, the regular-wiring speed-up the paper notes.
"""
from typing import List, Optional, Sequence, Tuple

from . import mle
from .circuit import MUL, Circuit
from .field import HALF, P, from_bytes
from .prover import combined_eq
from .transcript import TAG_DIGEST, TAG_VALUE, Transcript, circuit_digest, vector_digest


class MalformedProof(ValueError):
    pass


def interpolate(e: Sequence[int], r: int) -> int:
    """Value at r of the degree-2 polynomial with values e0, e1, e2 at 0, 1, 2."""
    e0, e1, e2 = e
    l0 = (r - 1) * (r - 2) % P * HALF
    l1 = -r * (r - 2)
    l2 = r * (r - 1) % P * HALF
    return (e0 * l0 + e1 * l1 + e2 * l2) % P


def predicates_generic(circuit: Circuit, i: int, u, v, alpha, beta, rx, ry) -> Tuple[int, int]:
    """(add~, mult~) at (r_x, r_y) weighted by T, from the flattened gate list."""
    T = combined_eq(u, v, alpha, beta)
    ex, ey = mle.eq_table(rx), mle.eq_table(ry)
    add_v = mul_v = 0
    for z, (x, y, t) in enumerate(circuit.flat_gates(i)):
        term = T[z] * ex[x] % P * ey[y]
        if t == MUL:
            mul_v += term
        else:
            add_v += term
    return add_v % P, mul_v % P


def _triple_eq(a: Sequence[int], b: Sequence[int], d: Sequence[int]) -> int:
    acc = 1
    for ak, bk, dk in zip(a, b, d):
        acc = acc * (ak * bk % P * dk + (1 - ak) * (1 - bk) % P * (1 - dk)) % P
    return acc


def predicates_factored(circuit: Circuit, i: int, u, v, alpha, beta, rx, ry) -> Tuple[int, int]:
    """(add~, mult~) using the sub-circuit once and the copy bits in closed form."""
    sg, sg1 = circuit.sigma[i], circuit.sigma[i + 1]
    elx, ely = mle.eq_table(rx[:sg1]), mle.eq_table(ry[:sg1])
    wu = mle.eq_table(u[:sg])
    cu = _triple_eq(u[sg:], rx[sg1:], ry[sg1:])
    if v is None:
        weight = [alpha * a % P * cu % P for a in wu]
    else:
        wv = mle.eq_table(v[:sg])
        cv = _triple_eq(v[sg:], rx[sg1:], ry[sg1:])
        weight = [(alpha * a % P * cu + beta * b % P * cv) % P for a, b in zip(wu, wv)]
    xs, ys, ts = circuit.wiring[i]
    add_v = mul_v = 0
    for z in range(1 << sg):
        term = weight[z] * elx[xs[z]] % P * ely[ys[z]]
        if ts[z] == MUL:
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


def _check_phase(rd: _Reader, nvars: int, claim: int, tr: Transcript):
    """Returns (ok, final claim, challenges)."""
    rs = []
    ok = True
    for _ in range(nvars):
        e = [rd.element(), rd.element(), rd.element()]
        if (e[0] + e[1]) % P != claim:
            ok = False
        r = tr.round_challenge(e[0], e[2])
        rs.append(r)
        claim = interpolate(e, r)
    return ok, claim, rs


def verify(circuit: Circuit, inputs: Sequence[int], outputs: Sequence[int], seed: int,
           proof: bytes, predicates=predicates_factored) -> bool:
    """True iff the proof convinces the verifier that outputs = circuit(inputs).

    Raises MalformedProof for a proof of the wrong length or a non-canonical element,
    and ValueError for input/output vectors of the wrong size or range.
    """
    d = circuit.depth
    if len(inputs) != 1 << circuit.s(d) or len(outputs) != 1 << circuit.s(0):
        raise ValueError("input or output vector has the wrong size")
    if any(not 0 <= a < P for a in inputs) or any(not 0 <= a < P for a in outputs):
        raise ValueError("input or output element not canonical")
    return _verify_core(circuit, seed, proof, predicates,
                        vector_digest(inputs), vector_digest(outputs),
                        lambda r: mle.evaluate(list(inputs), r),
                        lambda r: mle.evaluate(list(outputs), r))


def verify_limbs(circuit: Circuit, inputs_limbs, outputs_limbs, seed: int, proof: bytes,
                 predicates=predicates_factored) -> bool:
    """verify() for vectors given as canonical (count, 8) uint32 limb arrays.

    The statement digests hash the raw little-endian bytes (the canonical
    encoding) and the two large multilinear extensions use the C helper in
    oracle/fast.py; everything else is the same code as verify().
    """
    import numpy as np

    from . import fast
    from .transcript import tree_digest

    d = circuit.depth
    ins = np.ascontiguousarray(inputs_limbs, dtype=np.uint32)
    outs = np.ascontiguousarray(outputs_limbs, dtype=np.uint32)
    if ins.shape != (1 << circuit.s(d), 8) or outs.shape != (1 << circuit.s(0), 8):
        raise ValueError("input or output vector has the wrong size")
    top = P >> 224
    for arr in (ins, outs):
        if (arr[:, 7] > top).any():
            raise ValueError("input or output element not canonical")
    return _verify_core(circuit, seed, proof, predicates,
                        tree_digest(ins.tobytes()), tree_digest(outs.tobytes()),
                        lambda r: fast.mle_limbs(ins, r), lambda r: fast.mle_limbs(outs, r))


def _verify_core(circuit: Circuit, seed: int, proof: bytes, predicates, dig_in: bytes, dig_out: bytes,
                 mle_in, mle_out) -> bool:
    d = circuit.depth
    expected = sum((6 * circuit.s(i + 1) + 2) * 32 for i in range(d))
    if len(proof) != expected:
        raise MalformedProof("proof length %d, expected %d" % (len(proof), expected))
    rd = _Reader(proof)
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, circuit_digest(d, circuit.n, circuit.sigma, circuit.wiring))
    tr.absorb(TAG_DIGEST, dig_in)
    tr.absorb(TAG_DIGEST, dig_out)
    g = [tr.squeeze() for _ in range(circuit.s(0))]
    accept = True
    u: List[int] = g
    v: Optional[List[int]] = None
    vu, vv = mle_out(g), 0
    for i in range(d):
        if i == 0:
            alpha, beta = 1, 0
        else:
            alpha, beta = tr.squeeze(), tr.squeeze()
        claim = (alpha * vu + beta * vv) % P
        s1 = circuit.s(i + 1)
        ok1, claim, rx = _check_phase(rd, s1, claim, tr)
        vx = rd.element()
        tr.absorb_elements(TAG_VALUE, [vx])
        ok2, claim, ry = _check_phase(rd, s1, claim, tr)
        vy = rd.element()
        tr.absorb_elements(TAG_VALUE, [vy])
        add_v, mul_v = predicates(circuit, i, u, v, alpha, beta, rx, ry)
        final = (mul_v * vx % P * vy + add_v * (vx + vy)) % P
        accept = accept and ok1 and ok2 and final == claim
        u, v, vu, vv = rx, ry, vx, vy
    accept = accept and vu == mle_in(u) and vv == mle_in(v)
    return accept
