"""Fiat-Shamir transcript over SHA-256 (non-interactive form of the verifier's challenges).

In the paper the verifier sends a fresh random challenge after every round
message (Section 3.2.1). Here the challenges are derived from a SHA-256 hash
chain so a proof is a deterministic byte string:

  init           st = SHA256("SISU-GKR-v1" || LE64(seed))
  absorb(t, m)   st = SHA256(st || t || m), t a four-byte tag
  accept         v = LE(st) mod 2^254; while v >= p: st = SHA256(st || "GKRC"), v = LE(st) mod 2^254;
                 the challenge is v * 2^-256 mod p
  squeeze        st = SHA256(st || "GKRC"), then accept
  round(e0, e2)  st = C(st, LE(e0 * 2^256 mod p) || LE((e2 * 2^256 mod p) + 2^254)), then accept

C is the SHA-256 compression function (FIPS 180-4, Section 6.2.2) with st as
the chaining value and one 64-byte block: a round message costs one
compression. The challenge v * 2^-256 mod p is uniform on [0, p) like v (a
fixed bijection), and a round hashes e * 2^256 mod p (also a bijection of e);
both are the Montgomery representations (R = 2^256) a prover computing in
Montgomery form holds, so it hashes and takes challenges without
conversions. Both hashed values are below p < 2^254, so bit 254 of the
second one is free; it is set to mark a round block. Tags: "GKRD" statement digests,
"GKRV" a layer's final value, "GKRC" challenge rehashing. A round absorbs e0
and e2 only: e1 is fixed by the running claim (e1 = claim - e0, which the
verifier checks), so the state still binds the whole round polynomial; the
proof carries all three values. Tags are four bytes so that every absorbed
message stays word-aligned for SHA-256. Field elements are absorbed as
canonical 32-byte little-endian strings.

Statement digests (absorbed before any challenge):
  circuit  SHA256(LE32 d || LE32 n || LE32 sigma_0..sigma_d ||
                  for each gate layer, each gate z: LE32 x_z || LE32 y_z || u8 type_z)
  vectors  tree_digest of the canonical element bytes: split into 1 KiB
           chunks; a single chunk hashes directly, otherwise the
           concatenated chunk digests are digested again the same way.
"""
import hashlib
import struct
from typing import Sequence

from .field import P, encode_all, to_bytes

DOMAIN = b"SISU-GKR-v1"
CHUNK_BYTES = 1024
TAG_DIGEST = b"GKRD"
TAG_VALUE = b"GKRV"
TAG_CHALLENGE = b"GKRC"
_MASK254 = (1 << 254) - 1
_ROUND_MARK = 1 << 254
_R = (1 << 256) % P
_RINV = pow(1 << 256, -1, P)
_W32 = 0xFFFFFFFF


def _primes(count):
    out, k = [], 2
    while len(out) < count:
        if all(k % q for q in out if q * q <= k):
            out.append(k)
        k += 1
    return out


def _iroot(n, e):
    """floor(n^(1/e)) for an integer n >= 0."""
    lo, hi = 0, 1 << (n.bit_length() // e + 1)
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mid ** e <= n:
            lo = mid
        else:
            hi = mid - 1
    return lo


# FIPS 180-4 Section 4.2.2 / 5.3.3: the first 32 bits of the fractional parts
# of the cube roots of the first 64 primes, and of the square roots of the
# first 8 primes (computed here from that definition).
SHA256_K = [_iroot(q << 96, 3) & _W32 for q in _primes(64)]
SHA256_IV = [_iroot(q << 64, 2) & _W32 for q in _primes(8)]


def _rotr(x, n):
    return ((x >> n) | (x << (32 - n))) & _W32


def compress(state: bytes, block: bytes) -> bytes:
    """SHA-256 compression (FIPS 180-4 Section 6.2.2): chaining value `state`
    (32 bytes, big-endian words) and one 64-byte block."""
    assert len(state) == 32 and len(block) == 64
    H = struct.unpack(">8I", state)
    W = list(struct.unpack(">16I", block))
    for t in range(16, 64):
        s0 = _rotr(W[t - 15], 7) ^ _rotr(W[t - 15], 18) ^ (W[t - 15] >> 3)
        s1 = _rotr(W[t - 2], 17) ^ _rotr(W[t - 2], 19) ^ (W[t - 2] >> 10)
        W.append((W[t - 16] + s0 + W[t - 7] + s1) & _W32)
    a, b, c, d, e, f, g, h = H
    for t in range(64):
        t1 = (h + (_rotr(e, 6) ^ _rotr(e, 11) ^ _rotr(e, 25)) + ((e & f) ^ (~e & g)) + SHA256_K[t] + W[t]) & _W32
        t2 = ((_rotr(a, 2) ^ _rotr(a, 13) ^ _rotr(a, 22)) + ((a & b) ^ (a & c) ^ (b & c))) & _W32
        h, g, f, e, d, c, b, a = g, f, e, (d + t1) & _W32, c, b, a, (t1 + t2) & _W32
    return struct.pack(">8I", *((x + y) & _W32 for x, y in zip(H, (a, b, c, d, e, f, g, h))))


def sha256(data: bytes) -> bytes:
    return hashlib.sha256(data).digest()


def tree_digest(data: bytes) -> bytes:
    if len(data) <= CHUNK_BYTES:
        return sha256(data)
    level = b"".join(sha256(data[i:i + CHUNK_BYTES]) for i in range(0, len(data), CHUNK_BYTES))
    return tree_digest(level)


def vector_digest(values: Sequence[int]) -> bytes:
    return tree_digest(encode_all(values))


def circuit_digest(depth: int, log_copies: int, log_sub_width: Sequence[int], wiring) -> bytes:
    """wiring[i] = (x list, y list, type list) of gate layer i's sub-circuit."""
    parts = [struct.pack("<II", depth, log_copies)]
    parts += [struct.pack("<I", s) for s in log_sub_width]
    for xs, ys, ts in wiring:
        parts += [struct.pack("<IIB", int(x), int(y), int(t)) for x, y, t in zip(xs, ys, ts)]
    return sha256(b"".join(parts))


class Transcript:
    def __init__(self, seed: int):
        self.state = sha256(DOMAIN + struct.pack("<Q", seed & (2**64 - 1)))

    def absorb(self, tag: bytes, data: bytes) -> None:
        self.state = sha256(self.state + tag + data)

    def absorb_elements(self, tag: bytes, values: Sequence[int]) -> None:
        self.absorb(tag, b"".join(to_bytes(v) for v in values))

    def accept(self) -> int:
        """The current state as a challenge: rehash with "GKRC" until the
        254-bit value v is below p; the challenge is v * 2^-256 mod p."""
        v = int.from_bytes(self.state, "little") & _MASK254
        while v >= P:
            self.state = sha256(self.state + TAG_CHALLENGE)
            v = int.from_bytes(self.state, "little") & _MASK254
        return v * _RINV % P

    def squeeze(self) -> int:
        self.state = sha256(self.state + TAG_CHALLENGE)
        return self.accept()

    def round_challenge(self, e0: int, e2: int) -> int:
        """Absorb a round message (its values at t = 0 and t = 2) with one
        compression and return the challenge."""
        blk = to_bytes(e0 * _R % P) + ((e2 * _R % P) | _ROUND_MARK).to_bytes(32, "little")
        self.state = compress(self.state, blk)
        return self.accept()
