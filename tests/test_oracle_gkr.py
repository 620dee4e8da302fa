"""Pins of the oracle prover/verifier against definitions, brute force and invariants.

The brute-force checks recompute every round polynomial straight from the
GKR layer relation with multilinear predicates (no bookkeeping tables):
    f(x, y) = mult~_T(x, y) W~(x) W~(y) + add~_T(x, y) (W~(x) + W~(y)),
    mult~_T(x, y) = sum_{MUL z} T[z] eq(x, x_z) eq(y, y_z)   (add~_T over ADD gates),
so a dropped term, a wrong sign, a swapped operand or a wrong variable order in
the prover's tables fails them.
"""
import itertools
import random

import pytest

import gkr_synth as gs
from oracle import mle, prover, verifier
from oracle.circuit import ADD, MUL, Circuit, evaluate, evaluate_copy
from oracle.field import P
from oracle.transcript import Transcript

R = random.Random(2024)


def small_circuit(depth, n, sigmas, seed, mu=(1, 2)):
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=tuple(sigmas), mu=mu, seed=seed)
    c = Circuit.from_synth(spec, gs.make_wiring(spec))
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    return spec, c, inputs


def test_forward_by_hand():
    # 2 gates reading a 2-wide input layer: g0 = in0 * in1, g1 = in1 + in1
    c = Circuit(1, 0, [1, 1], [([0, 1], [1, 1], [MUL, ADD])])
    layers = evaluate(c, [3, 5])
    assert layers[0] == [15, 10]
    # with two copies: copy c reads inputs z*2+c
    c2 = Circuit(1, 1, [1, 1], [([0, 1], [1, 1], [MUL, ADD])])
    layers2 = evaluate(c2, [3, 4, 5, 6])  # copy0 = (3, 5), copy1 = (4, 6)
    assert layers2[0] == [15, 24, 10, 12]


def test_forward_matches_single_copy_evaluation():
    spec, c, inputs = small_circuit(3, 2, (3, 4, 2, 3), seed=11)
    layers = evaluate(c, inputs)
    n = c.n
    for cp in range(1 << n):
        mine = [inputs[(z << n) | cp] for z in range(1 << c.sigma[-1])]
        lay = evaluate_copy(c, mine)
        for i in range(c.depth + 1):
            assert lay[i] == [layers[i][(z << n) | cp] for z in range(1 << c.sigma[i])]


def _f(c: Circuit, i, T, W, x, y):
    gates = c.flat_gates(i)
    s1 = c.s(i + 1)
    wx, wy = mle.evaluate(W, x), mle.evaluate(W, y)
    acc = 0
    for z, (gx, gy, t) in enumerate(gates):
        w = T[z] * mle.eq(x, mle.bits_msb_first(gx, s1)) % P * mle.eq(y, mle.bits_msb_first(gy, s1)) % P
        acc += w * (wx * wy if t == MUL else wx + wy)
    return acc % P


def _cube(k):
    return [list(b) for b in itertools.product([0, 1], repeat=k)]


@pytest.mark.parametrize("shape", [
    (2, 0, (2, 2, 2), 1),
    (2, 1, (1, 2, 1), 2),
    (3, 1, (1, 1, 2, 1), 3),
    (1, 0, (0, 3), 4),
    (2, 2, (0, 1, 0), 5),
])
def test_round_polynomials_by_brute_force(shape):
    depth, n, sig, seed = shape
    spec, c, inputs = small_circuit(depth, n, sig, seed)
    layers = evaluate(c, inputs)
    pt = prover.prove_from_layers(c, layers, seed)
    u, v = pt.g, None
    for i, lt in enumerate(pt.layers):
        s1 = c.s(i + 1)
        W = layers[i + 1]
        T = prover.combined_eq(u, v, lt.alpha, lt.beta)
        # the phase-1 start claim is alpha V_i~(u) + beta V_i~(v)
        direct = (lt.alpha * mle.evaluate(layers[i], u)
                  + (lt.beta * mle.evaluate(layers[i], v) if v is not None else 0)) % P
        assert lt.claim == direct
        assert sum(_f(c, i, T, W, x, y) for x in _cube(s1) for y in _cube(s1)) % P == direct
        # phase 1
        for j, e in enumerate(lt.messages1):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, W, lt.rx[:j] + [t] + rest, y)
                            for rest in _cube(s1 - j - 1) for y in _cube(s1)) % P
                if t < 3:
                    assert e[t] == brute
                else:
                    assert verifier.interpolate(e, 3) == brute  # degree <= 2
        assert lt.vx == mle.evaluate(W, lt.rx)
        # phase 2
        for j, e in enumerate(lt.messages2):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, W, lt.rx, lt.ry[:j] + [t] + rest)
                            for rest in _cube(s1 - j - 1)) % P
                if t < 3:
                    assert e[t] == brute
                else:
                    assert verifier.interpolate(e, 3) == brute
        assert lt.vy == mle.evaluate(W, lt.ry)
        u, v = lt.rx, lt.ry


def test_round_invariant_and_final_predicate_check():
    spec, c, inputs = small_circuit(4, 3, (4, 3, 5, 2, 4), seed=21, mu=(3, 10))
    layers = evaluate(c, inputs)
    pt = prover.prove_from_layers(c, layers, 21)
    assert pt.claim0 == mle.evaluate(layers[0], pt.g)
    u, v = pt.g, None
    for i, lt in enumerate(pt.layers):
        claim = lt.claim
        for e, r in list(zip(lt.messages1, lt.rx)) + list(zip(lt.messages2, lt.ry)):
            assert (e[0] + e[1]) % P == claim
            claim = verifier.interpolate(e, r)
        a, m = verifier.predicates_generic(c, i, u, v, lt.alpha, lt.beta, lt.rx, lt.ry)
        a2, m2 = verifier.predicates_factored(c, i, u, v, lt.alpha, lt.beta, lt.rx, lt.ry)
        assert (a, m) == (a2, m2)
        assert claim == (m * lt.vx % P * lt.vy + a * (lt.vx + lt.vy)) % P
        u, v = lt.rx, lt.ry


@pytest.mark.parametrize("shape", [
    (4, 0, (10,) * 5, 1),
    (3, 3, (4, 5, 3, 4), 7),
    (2, 5, (0, 2, 1), 8),
    (1, 0, (0, 0), 9),
    (3, 2, (2, 0, 3, 1), 10),
])
def test_verifier_accepts_honest_proofs(shape):
    depth, n, sig, seed = shape
    spec, c, inputs = small_circuit(depth, n, sig, seed)
    pt = prover.prove(c, inputs, seed)
    pb = pt.proof_bytes()
    assert len(pb) == prover.proof_length(c)
    assert verifier.verify(c, inputs, pt.outputs, seed, pb)
    assert verifier.verify(c, inputs, pt.outputs, seed, pb, predicates=verifier.predicates_generic)


def test_every_proof_element_is_bound():
    spec, c, inputs = small_circuit(2, 1, (2, 1, 2), seed=31)
    pt = prover.prove(c, inputs, 31)
    pb = bytearray(pt.proof_bytes())
    for k in range(len(pb) // 32):
        bad = bytearray(pb)
        v = int.from_bytes(bad[32 * k:32 * k + 32], "little")
        bad[32 * k:32 * k + 32] = ((v + 1) % P).to_bytes(32, "little")
        assert not verifier.verify(c, inputs, pt.outputs, 31, bytes(bad)), k


def test_statement_tampering_is_rejected():
    spec, c, inputs = small_circuit(3, 2, (3, 3, 3, 3), seed=41)
    pt = prover.prove(c, inputs, 41)
    pb = pt.proof_bytes()
    outs = list(pt.outputs)
    outs[5] = (outs[5] + 1) % P
    assert not verifier.verify(c, inputs, outs, 41, pb)
    ins = list(inputs)
    ins[-1] = (ins[-1] + 1) % P
    assert not verifier.verify(c, ins, pt.outputs, 41, pb)
    assert not verifier.verify(c, inputs, pt.outputs, 42, pb)
    # a proof for false outputs, made honestly for them, is still rejected at the input check
    layers = evaluate(c, inputs)
    layers[0] = outs
    forged = prover.prove_from_layers(c, layers, 41).proof_bytes()
    assert not verifier.verify(c, inputs, outs, 41, forged)


def test_malformed_proofs_raise():
    spec, c, inputs = small_circuit(1, 0, (2, 2), seed=5)
    pt = prover.prove(c, inputs, 5)
    pb = pt.proof_bytes()
    with pytest.raises(verifier.MalformedProof):
        verifier.verify(c, inputs, pt.outputs, 5, pb[:-1])
    bad = bytearray(pb)
    bad[0:32] = P.to_bytes(32, "little")
    with pytest.raises(verifier.MalformedProof):
        verifier.verify(c, inputs, pt.outputs, 5, bytes(bad))


def test_copy_partial_messages_sum_to_the_global_message():
    """Per-worker partial polynomials add up to the master's (Section 3.2.1, deVirgo rounds)."""
    spec, c, inputs = small_circuit(2, 2, (3, 3, 3), seed=51)
    layers = evaluate(c, inputs)
    pt = prover.prove_from_layers(c, layers, 51)
    lt = pt.layers[0]
    n, sg1 = c.n, c.sigma[1]
    T = prover.combined_eq(pt.g, None, 1, 0)
    W = layers[1]
    G, H = [0] * len(W), [0] * len(W)
    for z, (x, y, t) in enumerate(c.flat_gates(0)):
        if t == MUL:
            G[x] += T[z] * W[y]
        else:
            G[x] += T[z]
            H[x] += T[z] * W[y]
    tabs = [list(W), [g % P for g in G], [h % P for h in H]]
    for j in range(sg1):  # local rounds only
        h = len(tabs[0]) // 2
        parts = []
        for cp in range(1 << n):
            e = [0, 0, 0]
            for b in range(cp, h, 1 << n):  # entries of copy cp
                for t in range(3):
                    wt, gt, ht = (X[b] + t * (X[b + h] - X[b]) for X in tabs)
                    e[t] += wt * gt + ht
            parts.append([a % P for a in e])
        assert [sum(p[t] for p in parts) % P for t in range(3)] == lt.messages1[j]
        tabs = [mle.fold(X, lt.rx[j]) for X in tabs]


def test_copy_bit_handoff_rebuilds_the_master_tables():
    """Sisu's distributed product sumcheck (Section 3.2.1): each worker's final table
    values after the local rounds form 2^n-entry tables on which the master finishes."""
    spec, c, inputs = small_circuit(1, 3, (2, 3), seed=61)
    layers = evaluate(c, inputs)
    pt = prover.prove_from_layers(c, layers, 61)
    lt = pt.layers[0]
    n, sg1 = c.n, c.sigma[1]
    T = prover.combined_eq(pt.g, None, 1, 0)
    W = layers[1]
    finals = []
    for cp in range(1 << n):
        # worker cp: its own sub-circuit tables over the local variables only
        Wc = [W[(x << n) | cp] for x in range(1 << sg1)]
        Gc, Hc = [0] * len(Wc), [0] * len(Wc)
        for z, (x, y, t) in enumerate(c.flat_gates(0)):
            if z & ((1 << n) - 1) != cp:
                continue
            if t == MUL:
                Gc[x >> n] += T[z] * W[y]
            else:
                Gc[x >> n] += T[z]
                Hc[x >> n] += T[z] * W[y]
        tabs = [Wc, [g % P for g in Gc], [h % P for h in Hc]]
        for j in range(sg1):
            tabs = [mle.fold(X, lt.rx[j]) for X in tabs]
        finals.append([X[0] for X in tabs])
    master = [[f[k] for f in finals] for k in range(3)]
    tr = Transcript(0)  # challenges are taken from the proof, not re-derived
    msgs = []
    for j in range(sg1, sg1 + n):
        h = len(master[0]) // 2
        e = []
        for t in range(3):
            acc = 0
            for b in range(h):
                wt, gt, ht = (X[b] + t * (X[b + h] - X[b]) for X in master)
                acc += wt * gt + ht
            e.append(acc % P)
        msgs.append(e)
        master = [mle.fold(X, lt.rx[j]) for X in master]
    assert msgs == lt.messages1[sg1:]
    assert master[0][0] == lt.vx
    del tr


def test_sharded_oracle_matches_unsharded():
    """Splitting the copies into 2^k shards and summing shard messages gives the same proof."""
    spec, c, inputs = small_circuit(2, 3, (2, 2, 2), seed=71)
    layers = evaluate(c, inputs)
    pt = prover.prove_from_layers(c, layers, 71)
    lt = pt.layers[1]
    W = layers[2]
    n, k = c.n, 1
    T = prover.combined_eq(pt.layers[0].rx, pt.layers[0].ry, lt.alpha, lt.beta)
    G, H = [0] * len(W), [0] * len(W)
    for z, (x, y, t) in enumerate(c.flat_gates(1)):
        if t == MUL:
            G[x] += T[z] * W[y]
        else:
            G[x] += T[z]
            H[x] += T[z] * W[y]
    tabs = [list(W), [g % P for g in G], [h % P for h in H]]
    shard_of = lambda b: (b & ((1 << n) - 1)) >> (n - k)  # top copy bit picks the shard
    for j in range(c.sigma[2]):
        h = len(tabs[0]) // 2
        sums = [[0, 0, 0] for _ in range(1 << k)]
        for b in range(h):
            for t in range(3):
                wt, gt, ht = (X[b] + t * (X[b + h] - X[b]) for X in tabs)
                sums[shard_of(b)][t] += wt * gt + ht
        assert [sum(s[t] for s in sums) % P for t in range(3)] == lt.messages1[j]
        tabs = [mle.fold(X, lt.rx[j]) for X in tabs]
