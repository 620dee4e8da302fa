"""Fiat-Shamir transcript over SHA-256 (non-interactive form of the verifier's challenges).

In the paper the verifier sends a fresh random challenge after every round
message (Section 3.2.1). Here the challenges are derived from a SHA-256 hash
chain so a proof is a deterministic byte string:

  init           st = SHA256("SISU-GKR-v1" || LE64(seed))
  absorb(t, m)   st = SHA256(st || t || m), t a four-byte tag
  accept         v = LE(st) mod 2^254; while v >= p: st = SHA256(st || "GKRC"), v = LE(st) mod 2^254
  squeeze        st = SHA256(st || "GKRC"), then accept
  round(e0, e2)  absorb("GKRR", e0 || e2), then accept: the round challenge

Tags: "GKRD" statement digests, "GKRR" a round message, "GKRV" a layer's
final value. A round absorbs e0 and e2 only: e1 is fixed by the running claim
(e1 = claim - e0, which the verifier checks), so the hash still binds the
whole round polynomial; the proof carries all three values. Tags are four
bytes so that every absorbed message stays word-aligned for SHA-256. Field
elements are absorbed as canonical 32-byte little-endian strings.

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
TAG_ROUND = b"GKRR"
TAG_VALUE = b"GKRV"
TAG_CHALLENGE = b"GKRC"
_MASK254 = (1 << 254) - 1


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
        """The current state as a challenge, rehashed with "GKRC" until below p."""
        v = int.from_bytes(self.state, "little") & _MASK254
        while v >= P:
            self.state = sha256(self.state + TAG_CHALLENGE)
            v = int.from_bytes(self.state, "little") & _MASK254
        return v

    def squeeze(self) -> int:
        self.state = sha256(self.state + TAG_CHALLENGE)
        return self.accept()

    def round_challenge(self, e0: int, e2: int) -> int:
        """Absorb a round message (its values at t = 0 and t = 2) and return the challenge."""
        self.absorb(TAG_ROUND, to_bytes(e0) + to_bytes(e2))
        return self.accept()
