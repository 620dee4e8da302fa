"""Pins of the SHA-256 transcript: FIPS 180-4 vectors, digest structure, determinism."""
import hashlib
import random
import struct

from oracle import field as F
from oracle import transcript as T


def test_sha256_fips_vectors():
    # FIPS 180-4 / NIST CSRC example values.
    assert T.sha256(b"abc").hex() == "ba7816bf8f01cfea414140de5dae2223b00361a396177a9cb410ff61f20015ad"
    assert T.sha256(b"").hex() == "e3b0c44298fc1c149afbf4c8996fb92427ae41e4649b934ca495991b7852b855"
    assert (T.sha256(b"abcdbcdecdefdefgefghfghighijhijkijkljklmklmnlmnomnopnopq").hex()
            == "248d6a61d20638b8e5c026930c3e6039a33ce45964ff2167f6ecedd419db06c1")


def test_tree_digest_structure():
    one = bytes(range(256)) * 4  # exactly one chunk
    assert len(one) == T.CHUNK_BYTES
    assert T.tree_digest(one) == hashlib.sha256(one).digest()
    two = one + b"\x07" * 100  # two chunks, the second short
    expect = hashlib.sha256(hashlib.sha256(one).digest() + hashlib.sha256(b"\x07" * 100).digest()).digest()
    assert T.tree_digest(two) == expect
    # CHUNK/32 + 1 leaves -> that many digests (one chunk plus 32 bytes) -> two digests -> root
    leaves = T.CHUNK_BYTES // 32 + 1
    big = b"\x01" * (T.CHUNK_BYTES * leaves)
    lvl1 = b"".join(hashlib.sha256(big[i:i + T.CHUNK_BYTES]).digest() for i in range(0, len(big), T.CHUNK_BYTES))
    assert len(lvl1) == T.CHUNK_BYTES + 32
    lvl2 = hashlib.sha256(lvl1[:T.CHUNK_BYTES]).digest() + hashlib.sha256(lvl1[T.CHUNK_BYTES:]).digest()
    assert T.tree_digest(big) == hashlib.sha256(lvl2).digest()


def test_transcript_chain_by_hand():
    tr = T.Transcript(5)
    st0 = hashlib.sha256(b"SISU-GKR-v1" + struct.pack("<Q", 5)).digest()
    assert tr.state == st0
    tr.absorb(b"GKRD", b"xyz")
    st1 = hashlib.sha256(st0 + b"GKRD" + b"xyz").digest()
    assert tr.state == st1
    v = tr.squeeze()
    st = st1
    while True:
        st = hashlib.sha256(st + b"GKRC").digest()
        cand = int.from_bytes(st, "little") % (1 << 254)
        if cand < F.P:
            break
    # the challenge is the accepted value times 2^-256 mod p
    assert v == cand * pow(2, -256, F.P) % F.P and tr.state == st


def _sha256_by_compression(msg: bytes) -> bytes:
    """SHA-256 through the oracle's compression function: FIPS 180-4 padding
    (Section 5.1.1) and the initial value, block by block."""
    pad = msg + b"\x80" + b"\x00" * ((55 - len(msg)) % 64) + (8 * len(msg)).to_bytes(8, "big")
    st = b"".join(v.to_bytes(4, "big") for v in T.SHA256_IV)
    for i in range(0, len(pad), 64):
        st = T.compress(st, pad[i:i + 64])
    return st


def test_compression_function_matches_hashlib():
    # the first constants as printed in FIPS 180-4
    assert T.SHA256_K[0] == 0x428A2F98 and T.SHA256_K[63] == 0xC67178F2
    assert T.SHA256_IV[0] == 0x6A09E667 and T.SHA256_IV[7] == 0x5BE0CD19
    rng = random.Random(5)
    for n in (0, 1, 3, 55, 56, 63, 64, 65, 119, 120, 128, 200, 1000):
        msg = bytes(rng.randrange(256) for _ in range(n))
        assert _sha256_by_compression(msg) == hashlib.sha256(msg).digest(), n


def test_round_challenge_by_hand():
    tr = T.Transcript(8)
    st = tr.state
    e0, e2 = 12345, F.P - 7
    r = tr.round_challenge(e0, e2)
    # one compression of the block LE(e0 2^256 mod p) || LE(e2 2^256 mod p) with bit 254 of the second set
    R = pow(2, 256, F.P)
    blk = (e0 * R % F.P).to_bytes(32, "little") + ((e2 * R % F.P) + (1 << 254)).to_bytes(32, "little")
    st = T.compress(st, blk)
    while int.from_bytes(st, "little") % (1 << 254) >= F.P:
        st = hashlib.sha256(st + b"GKRC").digest()
    v = int.from_bytes(st, "little") % (1 << 254)
    assert r * pow(2, 256, F.P) % F.P == v and tr.state == st
    # the challenge depends on both absorbed values
    t2 = T.Transcript(8)
    assert t2.round_challenge(e0, e2 - 1) != r
    t3 = T.Transcript(8)
    assert t3.round_challenge(e0 + 1, e2) != r


def test_squeeze_is_uniform_looking_and_in_range():
    tr = T.Transcript(99)
    vals = [tr.squeeze() for _ in range(400)]
    assert all(0 <= v < F.P for v in vals)
    assert len(set(vals)) == len(vals)
    # top bits are spread: about half of the values exceed P/2
    hi = sum(v > F.P // 2 for v in vals)
    assert 140 < hi < 260


def test_rejection_happens_at_the_expected_rate():
    # acceptance is P / 2^254 ~ 0.756; count SHA calls over many squeezes
    tr = T.Transcript(3)
    calls = 0
    for _ in range(2000):
        st = tr.state
        v = tr.squeeze()
        s, k = st, 0
        while True:
            s = hashlib.sha256(s + b"GKRC").digest()
            k += 1
            if int.from_bytes(s, "little") % (1 << 254) < F.P:
                break
        calls += k
    assert abs(2000 / calls - F.P / 2**254) < 0.03


def test_determinism_and_seed_sensitivity():
    a, b, c = T.Transcript(1), T.Transcript(1), T.Transcript(2)
    assert [a.squeeze() for _ in range(5)] == [b.squeeze() for _ in range(5)]
    assert T.Transcript(1).squeeze() != c.squeeze()


def test_circuit_digest_layout():
    wiring = [([1, 0], [0, 1], [1, 0])]
    d = T.circuit_digest(1, 2, [1, 1], wiring)
    raw = struct.pack("<IIII", 1, 2, 1, 1) + struct.pack("<IIB", 1, 0, 1) + struct.pack("<IIB", 0, 1, 0)
    assert d == hashlib.sha256(raw).digest()
