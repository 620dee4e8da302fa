"""Pins of the general-circuit oracle (accumulation gates, cross-layer inputs)
against definitions, brute force and invariants.

The brute-force checks recompute every round polynomial of a layer straight
from its relation with multilinear predicates, no bookkeeping tables:
    f(x, y') = sum over nested gates (g, x_r, y'_r) of T[g] eq(x, x_r) eq(y', y'_r)
               (W~(x) R~(y') for MUL, W~(x) + R~(y') for ADD),
where W = V_{i+1} and R~ is built from the source layers' values and the
used-gate index (Section 2.7), not from the prover's right-input vector.
"""
import itertools

import pytest

import gkr_synth as gs
from oracle import general as gen
from oracle import mle
from oracle.circuit import ADD, MUL, Circuit, evaluate as evaluate_layered
from oracle.field import P
from oracle.verifier import MalformedProof, interpolate


def _spec(depth, n, sig, seed, fanin=3, reach=3, cross=(1, 2), mu=(1, 2)):
    return gs.GeneralSpec(depth=depth, log_copies=n, log_sub_width=tuple(sig), max_fanin=fanin, reach=reach,
                          cross=cross, mu=mu, seed=seed)


def _case(spec):
    c = gen.GeneralCircuit.from_synth(spec, gs.make_general_wiring(spec))
    inputs = gs.elements_to_ints(gs.make_general_inputs(spec))
    return c, inputs


def test_accumulation_gate_adds_four_numbers_in_one_layer():
    """Section 3.4.3's example: one accumulation gate of two nested ADD gates
    sums four inputs in one layer (a layered circuit needs two layers)."""
    c = gen.GeneralCircuit(1, 0, [0, 2], [[(0, 0, 1, 1, ADD), (0, 2, 1, 3, ADD)]])
    assert gen.evaluate(c, [3, 5, 7, 11])[0] == [26]
    layered = Circuit(2, 0, [0, 1, 2], [([0], [1], [ADD]), ([0, 2], [1, 3], [ADD, ADD])])
    assert evaluate_layered(layered, [3, 5, 7, 11])[0] == [26]


def test_cross_layer_and_mixed_nested_gates_by_hand():
    # layer 1: z0 = a b, z1 = c + d; layer 0: (a b)(c + d) + (c + d) + a
    c = gen.GeneralCircuit(2, 0, [0, 1, 2], [
        [(0, 0, 1, 1, MUL), (0, 1, 2, 0, ADD)],
        [(0, 0, 2, 1, MUL), (1, 2, 2, 3, ADD)],
    ])
    a, b, cc, d = 3, 5, 7, 11
    layers = gen.evaluate(c, [a, b, cc, d])
    assert layers[1] == [a * b, cc + d]
    assert layers[0] == [a * b * (cc + d) + (cc + d) + a]
    assert c.sources[0] == [1, 2] and c.used[0] == {1: [1], 2: [0]}
    assert c.beta[0] == 1 and c.tau[0] == 0 and c.rho(0) == 1
    # with two copies every copy is evaluated alone
    c2 = gen.GeneralCircuit(2, 1, [0, 1, 2], c.records)
    ins = [a, 2, b, 4, cc, 6, d, 8]  # copy 0 = (a, b, c, d), copy 1 = (2, 4, 6, 8)
    assert gen.evaluate(c2, ins)[0] == [layers[0][0], 2 * 4 * (6 + 8) + (6 + 8) + 2]


def test_one_nested_gate_per_output_reading_the_next_layer_is_a_layered_circuit():
    spec = gs.CircuitSpec(depth=3, log_copies=2, log_sub_width=(3, 4, 2, 3), seed=5)
    wiring = gs.make_wiring(spec)
    lay = Circuit.from_synth(spec, wiring)
    recs = [[(z, int(w.x[z]), i + 1, int(w.y[z]), int(w.kind[z])) for z in range(len(w.x))]
            for i, w in enumerate(wiring)]
    c = gen.GeneralCircuit(spec.depth, spec.log_copies, spec.log_sub_width, recs)
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    assert gen.evaluate(c, inputs) == evaluate_layered(lay, inputs)


def test_right_vector_holds_the_used_gates_of_each_source():
    c, inputs = _case(_spec(4, 2, (2, 3, 3, 2, 3), seed=7))
    layers = gen.evaluate(c, inputs)
    n = c.n
    for i in range(c.depth):
        R = gen.right_vector(c, i, layers)
        assert len(R) == 1 << c.rho(i)
        filled = set()
        for z, x, j, y, t in c.records[i]:
            yl = c.right_index(i, j, y)
            for cp in range(1 << n):
                assert R[(yl << n) | cp] == layers[j][(y << n) | cp]
                filled.add((yl << n) | cp)
        assert all(R[k] == 0 for k in range(len(R)) if k not in filled)  # padding is zero


def _cube(k):
    return [list(b) for b in itertools.product([0, 1], repeat=k)]


def _r_mle(c, i, layers, point):
    """R_i~(point) from the source layers and the used-gate index, by definition."""
    n, tau = c.n, c.tau[i]
    acc = 0
    for b, j in enumerate(c.sources[i]):
        for k, y in enumerate(c.used[i][j]):
            for cp in range(1 << n):
                idx = (((b << tau) | k) << n) | cp
                acc += mle.eq(point, mle.bits_msb_first(idx, c.rho(i))) * layers[j][(y << n) | cp]
    return acc % P


def _f(c, i, T, layers, x, y):
    W = layers[i + 1]
    wx, ry = mle.evaluate(W, x), _r_mle(c, i, layers, y)
    s1, rho = c.s(i + 1), c.rho(i)
    acc = 0
    for g, xr, yr, t in c.flat_records(i):
        w = T[g] * mle.eq(x, mle.bits_msb_first(xr, s1)) % P * mle.eq(y, mle.bits_msb_first(yr, rho)) % P
        acc += w * (wx * ry if t == MUL else wx + ry)
    return acc % P


@pytest.mark.parametrize("shape", [
    (2, 0, (1, 2, 1), 1),
    (2, 1, (1, 1, 1), 2),
    (3, 0, (1, 1, 2, 1), 3),
    (1, 0, (0, 2), 4),
    (3, 1, (0, 1, 0, 1), 5),
])
def test_round_polynomials_by_brute_force(shape):
    depth, n, sig, seed = shape
    c, inputs = _case(_spec(depth, n, sig, seed))
    layers = gen.evaluate(c, inputs)
    pt = gen.prove_from_layers(c, layers, seed)
    # replay the claims in the order the prover produced them
    pending = [[] for _ in range(depth + 1)]
    pending[0].append(gen.Claim(0, "eq", pt.g, pt.claim0))
    for i, lt in enumerate(pt.layers):
        claims = pending[i]
        for cl in claims:  # every claim is true
            assert cl.value == sum(w * v for w, v in zip(gen.claim_weights(c, cl), layers[i])) % P
        T = gen.combined_weights(c, claims, lt.coefs)
        s1, rho = c.s(i + 1), c.rho(i)
        assert lt.claim == sum(a * b for a, b in zip(T, layers[i])) % P
        assert sum(_f(c, i, T, layers, x, y) for x in _cube(s1) for y in _cube(rho)) % P == lt.claim
        for j, e in enumerate(lt.messages1):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, layers, lt.rx[:j] + [t] + rest, y)
                            for rest in _cube(s1 - j - 1) for y in _cube(rho)) % P
                assert (e[t] if t < 3 else interpolate(e, 3)) == brute
        assert lt.vx == mle.evaluate(layers[i + 1], lt.rx)
        for j, e in enumerate(lt.messages2):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, layers, lt.rx, lt.ry[:j] + [t] + rest) for rest in _cube(rho - j - 1)) % P
                assert (e[t] if t < 3 else interpolate(e, 3)) == brute
        assert lt.vy == _r_mle(c, i, layers, lt.ry)
        # concatenation identity and each block value by definition
        beta = c.beta[i]
        eb = mle.eq_table(lt.ry[:beta])
        assert lt.vy == sum(e * v for e, v in zip(eb, lt.block_values)) % P
        for v, j in zip(lt.block_values, c.sources[i]):
            cl = gen.Claim(j, "subset", lt.ry[beta:], v, c.used[i][j])
            assert v == sum(w * a for w, a in zip(gen.claim_weights(c, cl), layers[j])) % P
        pending[i + 1].append(gen.Claim(i + 1, "eq", lt.rx, lt.vx))
        for v, j in zip(lt.block_values, c.sources[i]):
            pending[j].append(gen.Claim(j, "subset", lt.ry[beta:], v, c.used[i][j]))
    assert [(cl.kind, cl.value) for cl in pending[depth]] == [(cl.kind, cl.value) for cl in pt.input_claims]


@pytest.mark.parametrize("shape", [
    (2, 0, (2, 3, 2), 11),
    (4, 2, (2, 3, 3, 2, 3), 12),
    (3, 3, (0, 2, 1, 2), 13),
    (5, 1, (3, 3, 4, 3, 2, 3), 14),
])
def test_verifier_accepts_honest_proofs(shape):
    depth, n, sig, seed = shape
    c, inputs = _case(_spec(depth, n, sig, seed, fanin=4, reach=4))
    pt = gen.prove(c, inputs, seed)
    proof = pt.proof_bytes()
    assert len(proof) == gen.proof_length(c)
    assert gen.verify(c, inputs, pt.outputs, seed, proof)
    assert not gen.verify(c, inputs, pt.outputs, seed + 1, proof)


def test_every_proof_element_is_bound():
    c, inputs = _case(_spec(3, 1, (1, 2, 1, 2), seed=21, fanin=3))
    pt = gen.prove(c, inputs, 21)
    proof = pt.proof_bytes()
    for k in range(len(proof) // 32):
        bad = bytearray(proof)
        bad[32 * k] ^= 1
        try:
            ok = gen.verify(c, inputs, pt.outputs, 21, bytes(bad))
        except MalformedProof:
            ok = False
        assert not ok, "element %d is not checked" % k


def test_statement_tampering_is_rejected():
    c, inputs = _case(_spec(3, 1, (2, 2, 3, 2), seed=22))
    pt = gen.prove(c, inputs, 22)
    proof = pt.proof_bytes()
    outs = list(pt.outputs)
    outs[1] = (outs[1] + 1) % P
    assert not gen.verify(c, inputs, outs, 22, proof)
    ins = list(inputs)
    ins[-1] = (ins[-1] + 1) % P
    assert not gen.verify(c, ins, pt.outputs, 22, proof)
    # a different circuit (one nested gate's type flipped) binds a different statement
    recs = [list(r) for r in c.records]
    z, x, j, y, t = recs[1][0]
    recs[1][0] = (z, x, j, y, 1 - t)
    c2 = gen.GeneralCircuit(c.depth, c.n, c.sigma, recs)
    assert not gen.verify(c2, inputs, pt.outputs, 22, proof)
    with pytest.raises(MalformedProof):
        gen.verify(c, inputs, pt.outputs, 22, proof[:-32])


def test_planted_mistakes_fail_a_pin(monkeypatch):
    """A dropped ADD term in G, operands of phase 2 swapped, or the blocks of
    R_i out of order each break the brute-force check or the verifier."""
    c, inputs = _case(_spec(2, 1, (1, 2, 1), seed=31, fanin=3))
    layers = gen.evaluate(c, inputs)

    orig = gen.right_vector

    def broken_right_vector(c_, i, layers_):
        R = orig(c_, i, layers_)
        size = 1 << (c_.tau[i] + c_.n)
        return R[size:2 * size] + R[:size] + R[2 * size:]  # first two blocks swapped

    monkeypatch.setattr(gen, "right_vector", broken_right_vector)
    pt = gen.prove_from_layers(c, layers, 31)
    monkeypatch.setattr(gen, "right_vector", orig)
    assert len(c.sources[0]) >= 2
    assert not gen.verify(c, inputs, pt.outputs, 31, pt.proof_bytes())

    orig_fr = gen.GeneralCircuit.flat_records

    def swapped(self, i):  # phase tables built with x and y' exchanged on MUL gates
        return [(g, x, y, t) if t == ADD else (g, y % (1 << self.s(i + 1)), x % (1 << self.rho(i)), t)
                for g, x, y, t in orig_fr(self, i)]

    monkeypatch.setattr(gen.GeneralCircuit, "flat_records", swapped)
    pt2 = gen.prove_from_layers(c, layers, 31)
    monkeypatch.setattr(gen.GeneralCircuit, "flat_records", orig_fr)
    assert not gen.verify(c, inputs, pt2.outputs, 31, pt2.proof_bytes())


def test_digest_binds_every_field():
    c, _ = _case(_spec(2, 1, (1, 2, 1), seed=41))
    d0 = gen.digest(c)
    for layer in range(c.depth):
        for field in range(5):
            recs = [list(r) for r in c.records]
            r = list(recs[layer][0])
            if field == 2:
                continue  # the source layer must stay valid; changed below
            r[field] = r[field] ^ 1 if field != 4 else 1 - r[field]
            try:
                recs[layer][0] = tuple(r)
                c2 = gen.GeneralCircuit(c.depth, c.n, c.sigma, recs)
            except ValueError:
                continue
            assert gen.digest(c2) != d0
    assert gen.digest(gen.GeneralCircuit(c.depth, c.n + 1, c.sigma, c.records)) != d0
