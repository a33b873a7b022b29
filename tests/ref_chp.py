"""Independent pure stabilizer-tableau checker (Aaronson & Gottesman, PRA 70,
052328 (2004), "CHP"): 2n+1 rows, the g-function rowsum, and only the H, S,
CNOT primitives; every other Clifford is built from them.  Test code only.

Random measurement outcomes are decided from an explicit uniform u: outcome 0
iff u < 1/2 (a random Pauli measurement on a stabilizer state is 50/50).
"""
from __future__ import annotations


def _g(x1, z1, x2, z2):
    if x1 == 0 and z1 == 0:
        return 0
    if x1 == 1 and z1 == 1:
        return z2 - x2
    if x1 == 1 and z1 == 0:
        return z2 * (2 * x2 - 1)
    return x2 * (1 - 2 * z2)


class CHP:
    def __init__(self, n: int):
        self.n = n
        self.x = [0] * (2 * n + 1)
        self.z = [0] * (2 * n + 1)
        self.r = [0] * (2 * n + 1)
        for i in range(n):
            self.x[i] = 1 << i
            self.z[n + i] = 1 << i

    def _bit(self, w, q):
        return (w >> q) & 1

    def rowsum(self, h, i):
        tot = 2 * self.r[h] + 2 * self.r[i]
        for j in range(self.n):
            tot += _g(self._bit(self.x[i], j), self._bit(self.z[i], j),
                      self._bit(self.x[h], j), self._bit(self.z[h], j))
        # (for h = the pivot's own destabilizer the phase is odd and the row is
        # overwritten right after, as in the original algorithm)
        self.r[h] = 0 if tot % 4 == 0 else 1
        self.x[h] ^= self.x[i]
        self.z[h] ^= self.z[i]

    def h(self, a):
        for i in range(2 * self.n):
            xa, za = self._bit(self.x[i], a), self._bit(self.z[i], a)
            self.r[i] ^= xa & za
            if xa != za:
                self.x[i] ^= 1 << a
                self.z[i] ^= 1 << a

    def s(self, a):
        for i in range(2 * self.n):
            xa, za = self._bit(self.x[i], a), self._bit(self.z[i], a)
            self.r[i] ^= xa & za
            self.z[i] ^= xa << a

    def cnot(self, a, b):
        for i in range(2 * self.n):
            xa, za = self._bit(self.x[i], a), self._bit(self.z[i], a)
            xb, zb = self._bit(self.x[i], b), self._bit(self.z[i], b)
            self.r[i] ^= xa & zb & (xb ^ za ^ 1)
            self.x[i] ^= xa << b
            self.z[i] ^= zb << a

    # derived gates, from the primitives only
    def gate(self, name, *q):
        if name == "H":
            self.h(q[0])
        elif name == "S":
            self.s(q[0])
        elif name == "SDG":
            self.s(q[0]); self.s(q[0]); self.s(q[0])
        elif name == "Z":
            self.s(q[0]); self.s(q[0])
        elif name == "X":
            self.h(q[0]); self.s(q[0]); self.s(q[0]); self.h(q[0])
        elif name == "Y":
            self.gate("Z", q[0]); self.gate("X", q[0])
        elif name == "CX":
            self.cnot(q[0], q[1])
        elif name == "CZ":
            self.h(q[1]); self.cnot(q[0], q[1]); self.h(q[1])
        else:
            raise ValueError(name)

    def measure(self, a, u):
        n = self.n
        p = next((i for i in range(n, 2 * n) if self._bit(self.x[i], a)), None)
        if p is not None:
            for i in range(2 * n):
                if i != p and self._bit(self.x[i], a):
                    self.rowsum(i, p)
            self.x[p - n], self.z[p - n], self.r[p - n] = self.x[p], self.z[p], self.r[p]
            bit = 0 if u < 0.5 else 1
            self.x[p], self.z[p], self.r[p] = 0, 1 << a, bit
            return bit
        s = 2 * n
        self.x[s] = self.z[s] = self.r[s] = 0
        for i in range(n):
            if self._bit(self.x[i], a):
                self.rowsum(s, i + n)
        return self.r[s]


def run(text, meas_words):
    """Run a Clifford-only circuit.  Returns (chp, record)."""
    n = None
    sim = None
    record = []
    slot = 0
    for raw in text.splitlines():
        tok = raw.split("#")[0].split()
        if not tok:
            continue
        if tok[0] == "QUBITS":
            n = int(tok[1])
            sim = CHP(n)
            continue
        g = tok[0]
        if g in ("M", "R"):
            u = (float(meas_words[slot]) + 0.5) / 2.0 ** 32
            slot += 1
            bit = sim.measure(int(tok[1]), u)
            if g == "R":
                if bit:
                    sim.gate("X", int(tok[1]))
            else:
                record.append(bit)
        elif g in ("DETECTOR", "OBSERVABLE", "TICK"):
            pass
        else:
            sim.gate(g, *[int(t) for t in tok[1:]])
    return sim, record
