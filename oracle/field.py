"""Prime-field arithmetic for the oracle (BN254 scalar field, Section 4.1 "Choice of Finite Field").

The paper proves over BN254 for a pairing-friendly final verifier. The scalar
field Fr of BN254 has the prime below; elements are Python ints in [0, P).
"""

P = 21888242871839275222246405745257275088548364400416034343698204186575808495617
HALF = (P + 1) // 2  # inverse of 2
ELEMENT_BYTES = 32


def add(a: int, b: int) -> int:
    return (a + b) % P


def sub(a: int, b: int) -> int:
    return (a - b) % P


def mul(a: int, b: int) -> int:
    return (a * b) % P


def neg(a: int) -> int:
    return (-a) % P


def inv(a: int) -> int:
    """Multiplicative inverse by Fermat's little theorem."""
    if a % P == 0:
        raise ZeroDivisionError("inverse of zero")
    return pow(a, P - 2, P)


def to_bytes(a: int) -> bytes:
    """Canonical 32-byte little-endian encoding."""
    if not 0 <= a < P:
        raise ValueError("element not canonical")
    return a.to_bytes(ELEMENT_BYTES, "little")


def from_bytes(b: bytes) -> int:
    """Decode a 32-byte little-endian element; values >= P are malformed."""
    if len(b) != ELEMENT_BYTES:
        raise ValueError("element must be 32 bytes")
    v = int.from_bytes(b, "little")
    if v >= P:
        raise ValueError("element not canonical")
    return v


def encode_all(vals) -> bytes:
    return b"".join(to_bytes(v) for v in vals)
