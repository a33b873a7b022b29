"""Small seeded random circuits for the pins and parity tests (test code)."""
from __future__ import annotations

import numpy as np


def random_circuit(seed: int, n: int, length: int, p_t: float = 0.15, p_meas: float = 0.08,
                   p_mpp: float = 0.04, p_reset: float = 0.03, p_pauli: float = 0.08,
                   clifford_only: bool = False, allow_mpp: bool = True, gates=("H", "S", "SDG", "CX", "CZ"),
                   p_msc: float = 0.0, p_ccz: float = 0.0, p_diag: float = 0.0, p_if: float = 0.0):
    """Random circuit text and its measurement-slot count.  With p_msc > 0, a
    fraction p_msc of the ops come from the extended set: H_XY, H_NXY, MX,
    RX, MR, MRX and record-controlled Paulis XIF/YIF/ZIF; with p_ccz > 0 (and
    n >= 3) a fraction p_ccz are CCZ / CCX on three distinct qubits; with
    p_if > 0, a fraction p_if are classically controlled gates (IF) once a
    record exists."""
    rng = np.random.Generator(np.random.PCG64(seed))
    msc = rng if p_msc > 0 else None
    ccz = rng if p_ccz > 0 and n >= 3 else None
    dg = rng if p_diag > 0 else None
    cf = rng if p_if > 0 else None
    n_rec = 0
    if clifford_only:
        p_t = 0.0
    if not allow_mpp:
        p_mpp = 0.0
    lines = ["QUBITS %d" % n]
    n_meas_slots = 0
    for _ in range(length):
        if cf is not None and n_rec and cf.random() < p_if:
            lines.append(random_if(cf, n, n_rec))
            continue
        if dg is not None and dg.random() < p_diag:
            lines.append(random_diag(dg, n))
            continue
        if ccz is not None and ccz.random() < p_ccz:
            a, b, t = (int(x) for x in ccz.choice(n, size=3, replace=False))
            lines.append("%s %d %d %d" % ("CCZ" if ccz.integers(2) == 0 else "CCX", a, b, t))
            continue
        if msc is not None and msc.random() < p_msc:
            kind = int(msc.integers(7))
            q = int(msc.integers(n))
            if kind == 0:
                lines.append("%s %d" % ("H_XY" if msc.integers(2) == 0 else "H_NXY", q))
            elif kind <= 4:
                op = ("MX", "RX", "MR", "MRX")[kind - 1]
                lines.append("%s %d" % (op, q))
                n_meas_slots += 1
                n_rec += op != "RX"
            elif n_rec:
                lines.append("%sIF %d %d" % ("XYZ"[int(msc.integers(3))], int(msc.integers(n_rec)), q))
            continue
        u = rng.random()
        if u < p_t:
            lines.append("%s %d" % ("T" if rng.integers(2) == 0 else "TDG", rng.integers(n)))
        elif u < p_t + p_meas:
            lines.append("M %d" % rng.integers(n))
            n_meas_slots += 1
            n_rec += 1
        elif u < p_t + p_meas + p_mpp:
            k = int(rng.integers(1, n + 1))
            qs = rng.choice(n, size=k, replace=False)
            lines.append("MPP " + "*".join("%s%d" % ("XYZ"[rng.integers(3)], q) for q in qs))
            n_meas_slots += 1
            n_rec += 1
        elif u < p_t + p_meas + p_mpp + p_reset:
            lines.append("R %d" % rng.integers(n))
            n_meas_slots += 1
        elif u < p_t + p_meas + p_mpp + p_reset + p_pauli:
            lines.append("%s %d" % ("XYZ"[rng.integers(3)], rng.integers(n)))
        else:
            g = gates[int(rng.integers(len(gates)))]
            if g in ("CX", "CZ"):
                if n < 2:
                    continue
                a, b = rng.choice(n, size=2, replace=False)
                lines.append("%s %d %d" % (g, a, b))
            else:
                lines.append("%s %d" % (g, rng.integers(n)))
    return "\n".join(lines) + "\n", n_meas_slots


def random_diag(rng, n: int) -> str:
    """One diagonal gate: CS, CSDG, CPHASE, RZ, CCZ or a general DIAG on 1-3
    distinct qubits, angles drawn uniformly (printed exactly)."""
    kinds = ["RZ", "DIAG1"] + (["CS", "CSDG", "CPHASE", "DIAG2"] if n >= 2 else []) + (["CCZ", "DIAG3"] if n >= 3 else [])
    kind = kinds[int(rng.integers(len(kinds)))]
    ang = lambda: repr(float(rng.uniform(-np.pi, np.pi)))  # noqa: E731
    if kind.startswith("DIAG"):
        k = int(kind[4])
        qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
        return "DIAG %d %s %s" % (k, " ".join(map(str, qs)), " ".join(ang() for _ in range(1 << k)))
    if kind == "RZ":
        return "RZ %s %d" % (ang(), int(rng.integers(n)))
    if kind == "CCZ":
        return "CCZ %s" % " ".join(str(int(x)) for x in rng.choice(n, size=3, replace=False))
    a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
    return "CPHASE %s %d %d" % (ang(), a, b) if kind == "CPHASE" else "%s %d %d" % (kind, a, b)


def random_if(rng, n: int, n_rec: int) -> str:
    """One classically controlled gate: IF with the XOR of 1-3 record bits
    (repeats allowed, so some conditions cancel) or the AND of 2-3, on a
    Pauli, S, SDG, T, TDG, CZ or one of random_diag's gates."""
    k = int(rng.integers(1, 4))
    recs = [str(int(rng.integers(n_rec))) for _ in range(k)]
    cond = "&".join(recs) if (k > 1 and rng.integers(2) == 0) else ",".join(recs)
    u = int(rng.integers(6))
    q = int(rng.integers(n))
    if u == 0:
        gate = "%s %d" % ("XYZ"[int(rng.integers(3))], q)
    elif u == 1:
        gate = "%s %d" % (("S", "SDG", "T", "TDG")[int(rng.integers(4))], q)
    elif u == 2 and n >= 2:
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        gate = "CZ %d %d" % (a, b)
    elif u == 3 and n >= 3:
        gate = "CCX %s" % " ".join(str(int(x)) for x in rng.choice(n, size=3, replace=False))
    else:
        gate = random_diag(rng, n)
    return "IF %s %s" % (cond, gate)


def random_words(seed: int, count: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 1 << 32, size=count, dtype=np.uint64).astype(np.uint32)
