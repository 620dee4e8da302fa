"""Layered data-parallel circuits and their evaluation (GKR section, layer relation).

Layer 0 is the output layer and layer d the input layer. Layer i has
2^{s_i} gates; a fan-in-2 gate of layer i reads two gates x, y of layer i+1 and
outputs V_{i+1}(x) + V_{i+1}(y) (ADD) or V_{i+1}(x) * V_{i+1}(y) (MUL), which is
the paper's relation V_i(g) = sum add_i(g,x,y)(V(x)+V(y)) + mult_i(g,x,y)V(x)V(y)
with exactly one (x, y) pair connected to each g.

A data-parallel circuit is 2^n identical copies of one sub-circuit (the speed-up
noted at the end of the GKR section that the distributed prover of Section
3.2.1 relies on). Gate z of copy c is global gate g = z * 2^n + c and reads
global gates x_z * 2^n + c and y_z * 2^n + c.
"""
from typing import List, Sequence, Tuple

from .field import P

ADD = 0
MUL = 1


class Circuit:
    def __init__(self, depth: int, log_copies: int, log_sub_width: Sequence[int], wiring):
        """wiring[i] = (xs, ys, types) for the sub-circuit of gate layer i (length 2^{sigma_i})."""
        if depth < 1:
            raise ValueError("a circuit needs at least one gate layer")
        if len(log_sub_width) != depth + 1 or len(wiring) != depth:
            raise ValueError("shape mismatch")
        self.depth = depth
        self.n = log_copies
        self.sigma = [int(s) for s in log_sub_width]
        self.wiring: List[Tuple[List[int], List[int], List[int]]] = []
        for i, (xs, ys, ts) in enumerate(wiring):
            xs, ys, ts = [int(v) for v in xs], [int(v) for v in ys], [int(v) for v in ts]
            if not (len(xs) == len(ys) == len(ts) == 1 << self.sigma[i]):
                raise ValueError("layer %d has the wrong gate count" % i)
            lim = 1 << self.sigma[i + 1]
            if any(v >= lim for v in xs) or any(v >= lim for v in ys):
                raise ValueError("layer %d reads outside the next layer" % i)
            if any(t not in (ADD, MUL) for t in ts):
                raise ValueError("unknown gate type")
            self.wiring.append((xs, ys, ts))

    @classmethod
    def from_synth(cls, spec, wiring) -> "Circuit":
        return cls(spec.depth, spec.log_copies, spec.log_sub_width,
                   [(w.x.tolist(), w.y.tolist(), w.kind.tolist()) for w in wiring])

    def s(self, i: int) -> int:
        """log2 of the number of gates of layer i."""
        return self.sigma[i] + self.n

    def flat_gates(self, i: int) -> List[Tuple[int, int, int]]:
        """Global gate list of layer i: entry g = (x, y, type) with global indices."""
        xs, ys, ts = self.wiring[i]
        n = self.n
        out = [None] * (1 << self.s(i))
        for z in range(1 << self.sigma[i]):
            for c in range(1 << n):
                out[(z << n) | c] = ((xs[z] << n) | c, (ys[z] << n) | c, ts[z])
        return out

    def gate_layers(self) -> int:
        return sum(1 << self.s(i) for i in range(self.depth))


def evaluate_layer(circuit: Circuit, i: int, nxt: Sequence[int]) -> List[int]:
    """V_i from V_{i+1} (one gate at a time, from the definition)."""
    out = []
    for x, y, t in circuit.flat_gates(i):
        out.append((nxt[x] * nxt[y]) % P if t == MUL else (nxt[x] + nxt[y]) % P)
    return out


def evaluate(circuit: Circuit, inputs: Sequence[int]) -> List[List[int]]:
    """All layer values V_0 .. V_d, with V_d = inputs."""
    if len(inputs) != 1 << circuit.s(circuit.depth):
        raise ValueError("wrong input count")
    layers = [None] * (circuit.depth + 1)
    layers[circuit.depth] = list(inputs)
    for i in range(circuit.depth - 1, -1, -1):
        layers[i] = evaluate_layer(circuit, i, layers[i + 1])
    return layers


def evaluate_copy(circuit: Circuit, inputs_of_copy: Sequence[int]) -> List[List[int]]:
    """Evaluate one copy of the sub-circuit alone: layers of width 2^{sigma_i}."""
    layers = [None] * (circuit.depth + 1)
    layers[circuit.depth] = list(inputs_of_copy)
    for i in range(circuit.depth - 1, -1, -1):
        xs, ys, ts = circuit.wiring[i]
        nxt = layers[i + 1]
        layers[i] = [(nxt[x] * nxt[y]) % P if t == MUL else (nxt[x] + nxt[y]) % P
                     for x, y, t in zip(xs, ys, ts)]
    return layers
