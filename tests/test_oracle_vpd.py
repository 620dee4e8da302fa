"""Pins of the input-layer commitment oracle (oracle/vpd.py): every step is
checked against a definition it does not use itself (Horner evaluation,
schoolbook products, brute-force sums over the subgroup, hashlib), and the
verifier accepts honest openings and rejects tampered or cheating ones."""
import hashlib
import random
import struct

import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import mle, vpd
from oracle.field import P
from oracle.transcript import Transcript, compress
from oracle.verifier import MalformedProof


def rnd(rng, k):
    return [rng.randrange(P) for _ in range(k)]


# ---------------------------------------------------------------- field constants

def test_root_of_unity_has_order_two_to_the_28():
    w = vpd.ROOT_OF_UNITY
    assert pow(w, 1 << 28, P) == 1 and pow(w, 1 << 27, P) == P - 1
    assert (P - 1) % (1 << 28) == 0 and ((P - 1) >> 28) % 2 == 1      # 2-adicity exactly 28
    for m in (1, 2, 4, 1 << 10, 1 << 28):
        wm = vpd.root_of_unity(m)
        assert pow(wm, m, P) == 1
        if m > 1:
            assert pow(wm, m // 2, P) == P - 1


def test_coset_shift_is_outside_every_two_power_subgroup():
    # 5 is a quadratic non-residue and 5^(2^28) != 1: 5 <w_M> and <w_M> are disjoint
    assert pow(vpd.SHIFT, (P - 1) // 2, P) == P - 1
    assert pow(vpd.SHIFT, 1 << 28, P) != 1


def test_initial_hash_value_matches_hashlib():
    # one padded block of the empty message from the IV is SHA-256("")
    block = b"\x80" + bytes(63)
    assert compress(vpd.IV, block) == hashlib.sha256(b"").digest()


# ---------------------------------------------------------------- polynomials

@pytest.mark.parametrize("n", [1, 2, 8, 32])
def test_ntt_is_evaluation_on_the_subgroup(n):
    rng = random.Random(n)
    a = rnd(rng, n)
    w = vpd.root_of_unity(n)
    assert vpd.ntt(a, w) == [vpd.poly_eval(a, pow(w, k, P)) for k in range(n)]
    assert vpd.intt(vpd.ntt(a, w), w) == a


def test_poly_mul_matches_schoolbook():
    rng = random.Random(3)
    for la, lb in [(1, 1), (3, 5), (8, 8), (16, 7)]:
        a, b = rnd(rng, la), rnd(rng, lb)
        want = [0] * (la + lb - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                want[i + j] = (want[i + j] + x * y) % P
        assert vpd.poly_mul(a, b) == want


def test_bit_reversed_coset_table_positions():
    rng = random.Random(4)
    coeffs = rnd(rng, 4)
    m = 16
    tab = vpd.to_bitrev(vpd.coset_values(coeffs, m, vpd.SHIFT))
    for t in range(m):
        x = vpd.point_of_position(t, m, vpd.SHIFT)
        assert tab[t] == vpd.poly_eval(coeffs, x)
    for u in range(m // 2):
        # the pair (x, -x) is adjacent
        assert vpd.point_of_position(2 * u + 1, m, vpd.SHIFT) == (P - vpd.point_of_position(2 * u, m, vpd.SHIFT)) % P
    assert [vpd.bitrev(t, 3) for t in range(8)] == [0, 4, 2, 6, 1, 5, 3, 7]


@pytest.mark.parametrize("s", [0, 1, 3, 5])
def test_tensor_polynomial_is_the_eq_table_as_coefficients(s):
    rng = random.Random(10 + s)
    r = rnd(rng, s)
    table = mle.eq_table(r)
    for y in [0, 1, 2, rng.randrange(P)]:
        assert vpd.tensor_eval(r, y) == vpd.poly_eval(table, y)


def test_tensor_polynomial_splits_by_copy_bits():
    """The worker split of Section 3.2.2 on the tensor: with the copy bits
    last, Q_r(Y) = Q_{r_local}(Y^(2^n)) Q_{r_copy}(Y)."""
    rng = random.Random(12)
    r_loc, r_cp = rnd(rng, 3), rnd(rng, 2)
    y = rng.randrange(P)
    assert vpd.tensor_eval(r_loc + r_cp, y) == vpd.tensor_eval(r_loc, pow(y, 4, P)) * vpd.tensor_eval(r_cp, y) % P


@pytest.mark.parametrize("s", [0, 1, 2, 4])
def test_q_closed_form_matches_the_reversed_coefficients(s):
    rng = random.Random(20 + s)
    n = 1 << s
    r1, r2, lam = rnd(rng, s), rnd(rng, s), rng.randrange(P)
    w = [(a + lam * b) % P for a, b in zip(mle.eq_table(r1), mle.eq_table(r2))]
    q = [w[(n - j) % n] for j in range(n)]
    wn = vpd.root_of_unity(n)
    for x in [rng.randrange(P), vpd.SHIFT, pow(wn, 1 % n, P) if n > 1 else 1]:
        assert vpd.q_at(r1, r2, lam, x) == vpd.poly_eval(q, x)


@pytest.mark.parametrize("s", [0, 1, 3, 5])
def test_univariate_sumcheck_identity(s):
    """sum over H of f q = N (c1 + lam c2), brute force over the subgroup, and
    p = f q = c + X g' + (X^N - 1) h coefficient by coefficient."""
    rng = random.Random(30 + s)
    n = 1 << s
    V = rnd(rng, n)
    r1, r2, lam = rnd(rng, s), rnd(rng, s), rng.randrange(P)
    c = (mle.evaluate(V, r1) + lam * mle.evaluate(V, r2)) % P
    wn = vpd.root_of_unity(n)
    total = sum(vpd.poly_eval(V, pow(wn, k, P)) * vpd.q_at(r1, r2, lam, pow(wn, k, P)) for k in range(n)) % P
    assert total == n * c % P
    w = [(a + lam * b) % P for a, b in zip(mle.eq_table(r1), mle.eq_table(r2))]
    q = [w[(n - j) % n] for j in range(n)]
    gp, h = vpd.split_product(V, q, c)
    prod = [0] * (2 * n)
    for i, x in enumerate(V):
        for j, y in enumerate(q):
            prod[i + j] = (prod[i + j] + x * y) % P
    rebuilt = [0] * (2 * n)
    rebuilt[0] = c
    for k, v in enumerate(gp):
        rebuilt[k + 1] = (rebuilt[k + 1] + v) % P
    for k, v in enumerate(h):
        rebuilt[k + n] = (rebuilt[k + n] + v) % P
        rebuilt[k] = (rebuilt[k] - v) % P
    assert rebuilt == prod
    assert gp[-1] == 0 and h[-1] == 0           # deg g' <= N - 2, deg h <= N - 2
    with pytest.raises(ValueError):
        vpd.split_product(V, q, c + 1)


def test_fri_fold_matches_the_coefficient_fold():
    """Folding R(X) = E(X^2) + X O(X^2) by beta gives E + beta O on the squared coset."""
    rng = random.Random(40)
    coeffs = rnd(rng, 8)
    m, beta = 32, rng.randrange(P)
    tab = vpd.to_bitrev(vpd.coset_values(coeffs, m, vpd.SHIFT))
    folded = [(e + beta * o) % P for e, o in zip(coeffs[0::2], coeffs[1::2])]
    want = vpd.to_bitrev(vpd.coset_values(folded, m // 2, vpd.SHIFT * vpd.SHIFT % P))
    assert vpd.fold_table(tab, beta, vpd.SHIFT) == want


# ---------------------------------------------------------------- Merkle trees

def test_merkle_tree_by_hand():
    rng = random.Random(50)
    tab = rnd(rng, 8)
    tree = vpd.MerkleTree(vpd.pair_leaves(tab))
    mont = [(v * pow(2, 256, P) % P).to_bytes(32, "little") for v in tab]
    leaves = [vpd.chain(mont[2 * u] + mont[2 * u + 1]) for u in range(4)]
    n01 = compress(vpd.IV, leaves[0] + leaves[1])
    n23 = compress(vpd.IV, leaves[2] + leaves[3])
    assert tree.root == compress(vpd.IV, n01 + n23)
    assert tree.path(2) == [leaves[3], n01]
    for u in range(4):
        assert vpd.root_from_path(leaves[u], u, tree.path(u)) == tree.root
    assert vpd.root_from_path(leaves[1], 2, tree.path(2)) != tree.root


def test_chained_leaf_is_the_unpadded_compression_chain():
    # a 128-byte leaf: two compressions from the IV; hashlib's digest of the same
    # bytes differs only by its padding block
    data = bytes(range(128))
    st = compress(compress(vpd.IV, data[:64]), data[64:])
    assert vpd.chain(data) == st
    pad = b"\x80" + bytes(55) + struct.pack(">Q", 128 * 8)
    assert compress(st, pad) == hashlib.sha256(data).digest()


# ---------------------------------------------------------------- openings

def _claims(rng, s, V):
    r1, r2 = rnd(rng, s), rnd(rng, s)
    return r1, r2, mle.evaluate(V, r1), mle.evaluate(V, r2)


def _open(s, seed, queries=8):
    rng = random.Random(seed)
    V = rnd(rng, 1 << s)
    com = vpd.commit(V)
    r1, r2, c1, c2 = _claims(rng, s, V)
    op = vpd.open_at(com, r1, r2, c1, c2, Transcript(seed), queries)
    return com, r1, r2, c1, c2, op.proof_bytes()


def _verify(root, s, r1, r2, c1, c2, seed, pb, queries=8):
    try:
        return vpd.verify_opening(root, s, r1, r2, c1, c2, Transcript(seed), vpd._Reader(pb), queries)
    except MalformedProof:
        return False


@pytest.mark.parametrize("s", [0, 1, 2, 3, 6])
def test_honest_opening_accepted(s):
    com, r1, r2, c1, c2, pb = _open(s, 60 + s)
    assert len(pb) == vpd.opening_length(s, 8)
    assert _verify(com.root, s, r1, r2, c1, c2, 60 + s, pb)


def test_wrong_claims_rejected():
    s = 4
    com, r1, r2, c1, c2, pb = _open(s, 70)
    assert not _verify(com.root, s, r1, r2, (c1 + 1) % P, c2, 70, pb)
    assert not _verify(com.root, s, r1, r2, c1, (c2 + 1) % P, 70, pb)
    assert not _verify(com.root, s, r2, r1, c1, c2, 70, pb)
    other = vpd.commit([1] * (1 << s))
    assert not _verify(other.root, s, r1, r2, c1, c2, 70, pb)


def test_every_tampered_word_rejected():
    s = 3
    com, r1, r2, c1, c2, pb = _open(s, 80, queries=4)
    for off in range(0, len(pb), 32):
        bad = bytearray(pb)
        bad[off] ^= 1
        assert not _verify(com.root, s, r1, r2, c1, c2, 80, bytes(bad), 4), "word %d" % (off // 32)


def test_a_high_degree_table_is_caught():
    """A prover that commits to a table far from any polynomial of degree < N
    (a quarter of the positions replaced) and answers every query honestly from
    its tables is rejected: the folds stop being constant."""
    s = 5
    rng = random.Random(90)
    V = rnd(rng, 1 << s)
    com = vpd.commit(V)
    table = list(com.table)
    for t in rng.sample(range(len(table)), len(table) // 4):
        table[t] = rng.randrange(P)
    cheat = vpd.Commitment(com.coeffs, table, vpd.MerkleTree(vpd.pair_leaves(table)))
    r1, r2, c1, c2 = _claims(rng, s, V)
    with pytest.raises(ValueError):
        vpd.open_at(cheat, r1, r2, c1, c2, Transcript(90), 16)
    op = vpd.open_at(cheat, r1, r2, c1, c2, Transcript(90), 16, check_degree=False)
    assert not _verify(cheat.root, s, r1, r2, c1, c2, 90, op.proof_bytes(), 16)


def test_planted_mistakes_fail():
    """Plausible slips in the verifier's arithmetic each reject an honest opening."""
    s = 4
    com, r1, r2, c1, c2, pb = _open(s, 95)
    assert _verify(com.root, s, r1, r2, c1, c2, 95, pb)
    saved = vpd.q_at
    try:
        # q(x) taken as Q(1/x) off the subgroup (the (1 - x^N) Q(0) term dropped)
        vpd.q_at = lambda a, b, lam, x: (vpd.tensor_eval(a, pow(x, -1, P)) + lam * vpd.tensor_eval(b, pow(x, -1, P))) % P
        assert not _verify(com.root, s, r1, r2, c1, c2, 95, pb)
    finally:
        vpd.q_at = saved
    saved = vpd.point_of_position
    try:
        # natural-order positions instead of bit-reversed ones
        vpd.point_of_position = lambda t, m, shift: shift * pow(vpd.root_of_unity(m), t, P) % P
        assert not _verify(com.root, s, r1, r2, c1, c2, 95, pb)
    finally:
        vpd.point_of_position = saved
    saved = vpd._fold_pair
    try:
        # the odd part subtracted instead of added
        vpd._fold_pair = lambda pair, beta, x: ((pair[0] + pair[1]) * ((P + 1) // 2)
                                                - beta * (pair[0] - pair[1]) * ((P + 1) // 2) * pow(x, -1, P)) % P
        assert not _verify(com.root, s, r1, r2, c1, c2, 95, pb)
    finally:
        vpd._fold_pair = saved


# ---------------------------------------------------------------- GKR with a committed input layer

@pytest.mark.parametrize("depth,n,sig,seed", [(1, 0, (2, 3), 101), (3, 2, (3, 4, 3, 4), 102), (2, 3, (2, 1, 3), 103)])
def test_committed_gkr_proof(depth, n, sig, seed):
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=sig, mu=(1, 2), seed=seed)
    c = oc.Circuit.from_synth(spec, gs.make_wiring(spec))
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    pf = vpd.prove_committed(c, inputs, seed, queries=8)
    proof = pf.proof_bytes()
    assert len(proof) == vpd.committed_proof_length(c, 8)
    assert pf.outputs == oc.evaluate(c, inputs)[0]
    assert vpd.verify_committed(c, pf.outputs, seed, proof, 8)
    # the root is the commitment to the inputs
    assert proof[:32] == vpd.commit(inputs).root
    bad_out = list(pf.outputs)
    bad_out[0] = (bad_out[0] + 1) % P
    assert not vpd.verify_committed(c, bad_out, seed, proof, 8)
    gkr_end = 32 + sum((6 * c.s(i + 1) + 2) * 32 for i in range(depth))
    for off in (0, 32, gkr_end - 32, gkr_end, len(proof) - 32):
        bad = bytearray(proof)
        bad[off] ^= 1
        try:
            ok = vpd.verify_committed(c, pf.outputs, seed, bytes(bad), 8)
        except MalformedProof:
            ok = False
        assert not ok, "offset %d" % off
    with pytest.raises(MalformedProof):
        vpd.verify_committed(c, pf.outputs, seed, proof[:-32], 8)


def test_committed_proof_binds_the_inputs():
    """Proofs for two input vectors with the same outputs differ from the first byte:
    the commitment, not the outputs, fixes the transcript."""
    spec = gs.CircuitSpec(depth=1, log_copies=0, log_sub_width=(1, 2), mu=(0, 1), seed=7)
    c = oc.Circuit.from_synth(spec, gs.make_wiring(spec))
    a = [1, 2, 3, 4]
    pa = vpd.prove_committed(c, a, 7, queries=4)
    assert pa.root == vpd.commit(a).root and pa.root != vpd.commit([1, 2, 3, 5]).root
