"""Seeded synthetic circuit generators (inputs only).

These functions write circuit text in the format the sampler and the oracle
both parse.  They hold none of the simulation method: only circuit shapes,
random choices and GF(2) linear algebra for picking a CSS code.  Both the
tests and the benchmark draw their inputs from here.

The paper's workloads (magic state cultivation circuits, arXiv 2512.23037
Sec. III, Table II) are not available, so seed-generated circuits of the same
shape stand in for them:

* ``random_clifford_t``: 8 qubits, 200 gates uniform over {H, S, CNOT}, 6 T/T†
  and 8 mid-circuit Z measurements at uniform positions, half of them
  postselected on outcome 0.
* ``cultivation_shaped``: a random CSS code on the data qubits, |+> encoded,
  then "brackets" of a transversal T layer, a Z-check round, the inverse layer
  and an X-check round (every check postselected on 0), and a final logical X
  product measurement whose noiseless value is 0.  The Z checks commute with
  the diagonal T layer, so the noiseless pass rate is 1 (cf. Sec. IV-A: T on
  the data block only, Z-type constraints re-established between layers).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "random_clifford_t", "cultivation_shaped", "config", "mixture", "circuit_stats"]


@dataclass
class Workload:
    name: str
    text: str
    noise: dict
    seed: int
    meta: dict = field(default_factory=dict)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Random Clifford+T circuit (8 qubits, 200 Cliffords, 6 T/T†, 8 measurements)
# ---------------------------------------------------------------------------
def random_clifford_t(seed: int, n: int = 8, n_cliff: int = 200, n_t: int = 6, n_meas: int = 8,
                      n_post: int | None = None, p: float = 1e-3) -> Workload:
    rng = _rng(seed)
    if n_post is None:
        n_post = n_meas // 2
    kinds = ["C"] * n_cliff + ["T"] * n_t + ["M"] * n_meas
    order = rng.permutation(len(kinds))
    seq = [kinds[i] for i in order]
    post = set(rng.choice(n_meas, size=n_post, replace=False).tolist()) if n_meas else set()
    lines = ["QUBITS %d" % n]
    m_idx = 0
    for k in seq:
        if k == "C":
            g = int(rng.integers(3))
            if g == 0:
                lines.append("H %d" % rng.integers(n))
            elif g == 1:
                lines.append("S %d" % rng.integers(n))
            else:
                a, b = rng.choice(n, size=2, replace=False)
                lines.append("CX %d %d" % (a, b))
        elif k == "T":
            lines.append("%s %d" % ("T" if rng.integers(2) == 0 else "TDG", rng.integers(n)))
        else:
            lines.append("M %d" % rng.integers(n))
            if m_idx in post:
                lines.append("DETECTOR 0 %d" % m_idx)
            m_idx += 1
    # Gate noise only: DEP1 after every single-qubit gate, DEP2 after every CNOT.
    noise = {"p1": p, "p2": p}
    return Workload("random_clifford_t_n%d" % n, "\n".join(lines) + "\n", noise, seed,
                    {"n": n, "t_count": n_t, "measurements": n_meas})


# ---------------------------------------------------------------------------
# GF(2) helpers (code construction only)
# ---------------------------------------------------------------------------
def _rank(rows: list[int]) -> int:
    basis: dict[int, int] = {}
    for r in rows:
        while r:
            h = r.bit_length() - 1
            if h in basis:
                r ^= basis[h]
            else:
                basis[h] = r
                break
    return len(basis)


def _span(rows: list[int]) -> list[int]:
    out = [0]
    for r in rows:
        out += [x ^ r for x in out]
    return out


def _nullspace(rows: list[int], n: int) -> list[int]:
    """Basis of {x in GF(2)^n : popcount(x & r) even for every r}."""
    sols = []
    # Gaussian elimination on the n x n system, columns = coordinates.
    m = [r for r in rows]
    pivots = []
    mat = []
    for r in m:
        for (pc, pr) in zip(pivots, mat):
            if (r >> pc) & 1:
                r ^= pr
        if r:
            pc = r.bit_length() - 1
            # reduce existing rows
            for i in range(len(mat)):
                if (mat[i] >> pc) & 1:
                    mat[i] ^= r
            pivots.append(pc)
            mat.append(r)
    free = [c for c in range(n) if c not in pivots]
    for f in free:
        x = 1 << f
        for pc, pr in zip(pivots, mat):
            if (pr >> f) & 1:
                x |= 1 << pc
        sols.append(x)
    return sols


def _bits(x: int) -> list[int]:
    return [i for i in range(x.bit_length()) if (x >> i) & 1]


def _low_weight_basis(space: list[int], want: int, rng: np.random.Generator, exclude_span: list[int] = ()) -> list[int]:
    """Pick `want` independent low-weight vectors from a small linear space,
    independent of `exclude_span`; ties broken by the seeded generator."""
    cand = [v for v in space if v]
    keys = rng.random(len(cand))
    cand = [v for _, v in sorted(zip([(bin(v).count("1"), k) for v, k in zip(cand, keys)], cand))]
    chosen: list[int] = []
    base = list(exclude_span)
    r0 = _rank(base)
    for v in cand:
        if _rank(base + chosen + [v]) == r0 + len(chosen) + 1:
            chosen.append(v)
            if len(chosen) == want:
                break
    if len(chosen) < want:
        raise ValueError("not enough independent vectors")
    return chosen


def _layers(pairs: list[tuple[int, int]]) -> list[list[tuple[int, int]]]:
    """Greedy moments of gates on disjoint qubits, keeping the given order."""
    out: list[list[tuple[int, int]]] = []
    busy: list[set] = []
    for a, b in pairs:
        placed = False
        # earliest layer after the last layer touching a or b
        last = -1
        for i, s in enumerate(busy):
            if a in s or b in s:
                last = i
        i = last + 1
        if i < len(out):
            out[i].append((a, b))
            busy[i].update((a, b))
            placed = True
        if not placed:
            out.append([(a, b)])
            busy.append({a, b})
    return out


# ---------------------------------------------------------------------------
# Cultivation-shaped circuit family
# ---------------------------------------------------------------------------
def cultivation_shaped(seed: int, n_data: int, n_anc: int, r_z: int, brackets: list[int],
                       z_per_round: int | None = None, check_weight: int = 6, p: float = 1e-3,
                       name: str | None = None, inverse_order: str = "same") -> Workload:
    """Data qubits 0..n_data-1, ancillas after them.  ``brackets`` lists the
    size of each T layer (the first one of size n_data is transversal).
    ``inverse_order``: "same" writes each inverse layer in the order of its
    layer; "shuffled" in a seeded random order; "shuffled_tick" also puts a
    TICK (idle noise on the qubits not yet touched) in its middle."""
    rng = _rng(seed)
    r_x = n_data - 1 - r_z
    full = (1 << n_data) - 1
    # Z checks: random full-rank rows of weight `check_weight`.
    hz: list[int] = []
    while len(hz) < r_z:
        v = 0
        for q in rng.choice(n_data, size=min(check_weight, n_data), replace=False):
            v |= 1 << int(q)
        if _rank(hz + [v]) == len(hz) + 1:
            hz.append(v)
    null_z = _nullspace(hz, n_data)            # dim r_x + 1: X checks and logical X
    space = _span(null_z)
    hx = _low_weight_basis(space, r_x, rng)
    xbar = _low_weight_basis(space, 1, rng, exclude_span=hx)[0]
    assert all(bin(a & b).count("1") % 2 == 0 for a in hx + [xbar] for b in hz)
    if z_per_round is None:
        z_per_round = (n_anc + 1) // 2
    x_per_round = n_anc - z_per_round
    z_span = [v for v in _span(hz) if v]
    x_span = [v for v in _span(hx) if v]

    def round_checks(gens: list[int], span: list[int], count: int) -> list[int]:
        checks = list(gens)[:count]
        extra = count - len(checks)
        if extra > 0:
            w = np.array([bin(v).count("1") for v in span], dtype=float)
            prob = np.exp(-(w - w.min()))
            prob /= prob.sum()
            picks = rng.choice(len(span), size=extra, replace=True, p=prob)
            checks += [span[i] for i in picks]
        return checks

    # Encoder for |+>_L: rows of [H_X; Xbar] in reduced echelon form; H on the
    # pivot columns, CNOT from each pivot to the rest of its row.
    gen = hx + [xbar]
    mat: list[int] = []
    piv: list[int] = []
    for r in gen:
        for pc, pr in zip(piv, mat):
            if (r >> pc) & 1:
                r ^= pr
        assert r
        pc = r.bit_length() - 1
        for i in range(len(mat)):
            if (mat[i] >> pc) & 1:
                mat[i] ^= r
        piv.append(pc)
        mat.append(r)
    anc = list(range(n_data, n_data + n_anc))
    lines = ["QUBITS %d" % (n_data + n_anc)]
    rec = 0

    def emit_layers(pairs):
        for layer in _layers(pairs):
            for a, b in layer:
                lines.append("CX %d %d" % (a, b))
            lines.append("TICK")

    lines += ["H %d" % q for q in piv] + ["TICK"]
    enc = [(pc, q) for pc, pr in zip(piv, mat) for q in _bits(pr) if q != pc]
    enc = [enc[i] for i in rng.permutation(len(enc))]
    emit_layers(enc)

    t_layers = []
    for bi, size in enumerate(brackets):
        Q = list(range(n_data)) if size >= n_data else sorted(int(q) for q in rng.choice(n_data, size=size, replace=False))
        t_layers.append(Q)
        first, second = ("T", "TDG") if rng.integers(2) == 0 else ("TDG", "T")
        lines += ["%s %d" % (first, q) for q in Q] + ["TICK"]
        # Z-check round: CNOT data -> ancilla, measure, postselect 0, reset.
        zc = round_checks(hz, z_span, z_per_round)
        za = anc[:z_per_round]
        pairs = [(q, a) for a, h in zip(za, zc) for q in _bits(h)]
        pairs = [pairs[i] for i in rng.permutation(len(pairs))]
        emit_layers(pairs)
        for a in za:
            lines.append("M %d" % a)
            lines.append("DETECTOR 0 %d" % rec)
            rec += 1
        lines.append("TICK")
        lines += ["R %d" % a for a in za] + ["TICK"]
        inv = list(Q)
        if inverse_order != "same":
            inv = [inv[i] for i in rng.permutation(len(inv))]
        inv_lines = ["%s %d" % (second, q) for q in inv]
        if inverse_order == "shuffled_tick":
            inv_lines.insert(len(inv_lines) // 2, "TICK")
        lines += inv_lines + ["TICK"]
        # X-check round: ancilla in |+>, CNOT ancilla -> data, H, measure.
        xc = round_checks(hx, x_span, x_per_round)
        xa = anc[z_per_round:z_per_round + x_per_round]
        lines += ["H %d" % a for a in xa] + ["TICK"]
        pairs = [(a, q) for a, g in zip(xa, xc) for q in _bits(g)]
        pairs = [pairs[i] for i in rng.permutation(len(pairs))]
        emit_layers(pairs)
        lines += ["H %d" % a for a in xa] + ["TICK"]
        for a in xa:
            lines.append("M %d" % a)
            lines.append("DETECTOR 0 %d" % rec)
            rec += 1
        lines.append("TICK")
        lines += ["R %d" % a for a in xa] + ["TICK"]
    lines.append("MPP " + "*".join("X%d" % q for q in _bits(xbar)))
    lines.append("OBSERVABLE 0 %d" % rec)
    noise = {"p1": p, "p2": p, "p_idle": p, "p_meas": p, "p_reset": p, "p_mpp": p}
    meta = {"n_data": n_data, "n_anc": n_anc, "r_z": r_z, "r_x": r_x, "brackets": brackets,
            "hz": hz, "hx": hx, "xbar": xbar, "t_layers": t_layers}
    return Workload(name or "cultivation_shaped_%dq_%dT" % (n_data + n_anc, 2 * sum(len(q) for q in t_layers)),
                    "\n".join(lines) + "\n", noise, seed, meta)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def config(name: str, seed: int = 1, p: float | None = None) -> Workload:
    """Workloads by name:
    ``clifford_t_8q``   -- 8 qubits, 200 Cliffords, 6 T/T†, 8 measurements (p=1e-3)
    ``cultivation_15q`` -- 7 data + 8 ancilla, two transversal brackets (28 T/T†)
    ``cultivation_42q`` -- 19 data + 23 ancilla, brackets 19+7+5+5 (72 T/T†)
    ``cultivation_42q_k12`` -- the same family with 7 Z checks: support up to 2^12
    """
    if name == "clifford_t_8q":
        return random_clifford_t(seed, p=1e-3 if p is None else p)
    if name == "cultivation_15q":
        return cultivation_shaped(seed, 7, 8, 3, [7, 7], check_weight=4, p=1e-3 if p is None else p,
                                  name="cultivation_15q_28T")
    if name == "cultivation_42q":
        return cultivation_shaped(seed, 19, 23, 9, [19, 7, 5, 5], check_weight=6, p=1e-3 if p is None else p,
                                  name="cultivation_42q_72T")
    if name == "cultivation_42q_k12":
        return cultivation_shaped(seed, 19, 23, 7, [19, 7, 5, 5], check_weight=6, p=1e-3 if p is None else p,
                                  name="cultivation_42q_72T_k12")
    raise KeyError(name)


# The eight generated companions of the 15-qubit circuit in the mixed run:
# (data qubits, ancillas, Z-check rank, bracket sizes).  Qubits 12..20, 16..40
# T/T-dagger; the 12- and 13-data-qubit codes reach span dimension 10.
MIX_SHAPES = [(9, 5, 3, [9]), (10, 6, 3, [10, 4]), (11, 7, 3, [11, 5]), (12, 8, 2, [12, 4]),
              (8, 4, 3, [8, 8]), (13, 7, 3, [13, 7]), (10, 8, 4, [10, 5, 3]), (9, 7, 2, [9])]
MIX_P = (5e-4, 1e-3, 2e-3)


def mixture(seed: int = 1, total_shots: int = 10_000_000) -> dict:
    """Many circuits in one launch: the 15-qubit cultivation circuit plus the
    eight shapes of MIX_SHAPES, each at every p of MIX_P (27 variants), with
    the shots split evenly into consecutive global ranges.  Returns the
    variants' workloads, their noise dicts and the exclusive range ends."""
    circuits = [config("cultivation_15q", seed=seed)]
    for i, (nd, na, rz, br) in enumerate(MIX_SHAPES):
        circuits.append(cultivation_shaped(seed * 1000 + i, nd, na, rz, br, check_weight=min(5, nd - 2),
                                           name="mix%d_%dq_%dT" % (i, nd + na, 2 * sum(min(b, nd) for b in br))))
    works, models = [], []
    for w in circuits:
        for p in MIX_P:
            works.append(w)
            models.append({k: p for k in ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")})
    nv = len(works)
    ends = [total_shots * (v + 1) // nv for v in range(nv)]
    return {"workloads": works, "models": models, "shot_ends": ends}


def circuit_stats(text: str) -> dict:
    """Table II style statistics of a circuit text (noise ops excluded)."""
    n = 0
    gates = two_q = meas = tcount = 0
    tsupport: set = set()
    depth_at: list[int] = []
    tdepth_at: list[int] = []
    for raw in text.splitlines():
        tok = raw.split("#")[0].split()
        if not tok:
            continue
        op = tok[0]
        if op == "QUBITS":
            n = int(tok[1])
            depth_at = [0] * n
            tdepth_at = [0] * n
            continue
        if op in ("H", "S", "SDG", "X", "Y", "Z", "T", "TDG", "CX", "CZ", "M", "R", "MPP"):
            if op == "MPP":
                qs = [int(f[1:]) for f in tok[1].split("*")]
            else:
                qs = [int(x) for x in tok[1:]]
            gates += 1
            if len(qs) == 2 and op in ("CX", "CZ"):
                two_q += 1
            if op in ("M", "MPP"):
                meas += 1
            d = max(depth_at[q] for q in qs) + 1
            for q in qs:
                depth_at[q] = d
            if op in ("T", "TDG"):
                tcount += 1
                tsupport.add(qs[0])
                td = max(tdepth_at[q] for q in qs) + 1
                for q in qs:
                    tdepth_at[q] = td
            else:
                # T depth counts T layers along each qubit's history
                td = max(tdepth_at[q] for q in qs)
                for q in qs:
                    tdepth_at[q] = td
    return {"qubits": n, "gates": gates, "depth": max(depth_at) if depth_at else 0, "two_qubit_gates": two_q,
            "measurements": meas, "t_count": tcount, "t_support": len(tsupport),
            "t_depth": max(tdepth_at) if tdepth_at else 0}
