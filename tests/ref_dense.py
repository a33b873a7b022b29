"""Dense statevector checker for the oracle (test code, numpy, <= ~12 qubits).

It runs a circuit on a plain 2^n statevector with the textbook gate matrices
(H, S = diag(1, i), T = diag(1, e^{i pi/4}), CNOT, CZ, Paulis, (X +- Y)/sqrt2)
and, beside it,
a "shadow" copy of the stabilizer state |psi_S> whose global phase follows the
same reading the oracle uses: Cliffords and Paulis act on it as matrices, T
leaves it alone, and a measurement that is random on |psi_S> replaces it by
sqrt(2) Pi_m |psi_S>.  With the shadow, a generalized-stabilizer state
(tableau, v) can be expanded as sum_alpha v_alpha d_alpha |psi_S>
(Definition 1) and compared with the statevector with no global-phase freedom.

Measurement outcomes are decided here from the same explicit uniforms the
oracle receives (outcome +1 iff u < P(+1)), so the records are an independent
check too.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(0.5)
MATS = {
    "H": np.array([[1, 1], [1, -1]], dtype=complex) * SQ2,
    "S": np.diag([1, 1j]).astype(complex),
    "SDG": np.diag([1, -1j]).astype(complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.diag([1, -1]).astype(complex),
    "T": np.diag([1, np.exp(1j * np.pi / 4)]),
    "TDG": np.diag([1, np.exp(-1j * np.pi / 4)]),
    "H_XY": np.array([[0, 1 - 1j], [1 + 1j, 0]], dtype=complex) * SQ2,   # (X + Y)/sqrt2
    "H_NXY": np.array([[0, 1 + 1j], [1 - 1j, 0]], dtype=complex) * SQ2,  # (X - Y)/sqrt2
}


def popcount(a):
    return np.bitwise_count(np.asarray(a, dtype=np.uint64)).astype(np.int64)


def apply_1q(psi, U, q, n):
    t = psi.reshape([2] * n)
    ax = n - 1 - q
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [ax])), 0, ax)
    return t.reshape(-1)


def apply_cx(psi, a, b, n):
    idx = np.arange(1 << n, dtype=np.uint64)
    src = idx ^ (((idx >> np.uint64(a)) & np.uint64(1)) << np.uint64(b))
    return psi[src]


def apply_cz(psi, a, b, n):
    idx = np.arange(1 << n, dtype=np.uint64)
    ph = ((idx >> np.uint64(a)) & (idx >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return psi * (1 - 2 * ph)


def pauli_apply(psi, x, z, e, n):
    """Apply i^e (x) sigma(x_j, z_j) with sigma(1,1) = Y = i X Z."""
    idx = np.arange(1 << n, dtype=np.uint64)
    j = idx ^ np.uint64(x)
    sign = 1 - 2 * (popcount(j & np.uint64(z)) & 1)
    phase = 1j ** ((e + bin(x & z).count("1")) % 4)
    return phase * sign * psi[j]


def expval(psi, x, z, e, n):
    return np.vdot(psi, pauli_apply(psi, x, z, e, n))


def parse(text):
    ops = []
    n = None
    for raw in text.splitlines():
        tok = raw.split("#")[0].split()
        if not tok:
            continue
        if tok[0] == "QUBITS":
            n = int(tok[1])
            continue
        ops.append(tok)
    return n, ops


def mpp_pauli(spec):
    x = z = 0
    for f in spec.split("*"):
        q = int(f[1:])
        if f[0] in "XY":
            x |= 1 << q
        if f[0] in "ZY":
            z |= 1 << q
    return x, z


def run(text, meas_words):
    """Run a noiseless circuit (explicit Paulis allowed) on a statevector.

    Returns (phi, shadow, record, p0_list) where p0_list[k] = P(+1) at
    measurement slot k.  DETECTOR/OBSERVABLE lines are ignored."""
    n, ops = parse(text)
    phi = np.zeros(1 << n, dtype=complex)
    phi[0] = 1
    shadow = phi.copy()
    record = []
    p0s = []
    slot = 0
    for tok in ops:
        g = tok[0]
        if g == "IF":
            # classically controlled gate: XOR ("a,b") or AND ("a&b") of record
            # bits.  A Pauli updates the shadow as a bare Pauli does; a diagonal
            # gate (S, SDG, T, TDG, CZ or a DIAG-family gate) is applied to phi
            # only, its matrix written out here.
            cs = tok[1]
            bits = [record[int(r)] for r in cs.replace("&", ",").split(",")]
            fire = all(bits) if "&" in cs else (sum(bits) % 2 == 1)
            sub = tok[2:]
            if not fire:
                continue
            if sub[0] in ("X", "Y", "Z"):
                q = int(sub[1])
                phi = apply_1q(phi, MATS[sub[0]], q, n)
                shadow = apply_1q(shadow, MATS[sub[0]], q, n)
                continue
            if sub[0] in ("S", "SDG", "T", "TDG"):
                ph = {"S": np.pi / 2, "SDG": -np.pi / 2, "T": np.pi / 4, "TDG": -np.pi / 4}[sub[0]]
                phi = apply_1q(phi, np.diag([1.0, np.exp(1j * ph)]), int(sub[1]), n)
                continue
            if sub[0] == "CZ":
                phi = apply_cz(phi, int(sub[1]), int(sub[2]), n)
                continue
            if sub[0] in ("CCZ", "CCX"):
                a, b, t = int(sub[1]), int(sub[2]), int(sub[3])
                idx = np.arange(1 << n, dtype=np.uint64)
                on = ((idx >> np.uint64(a)) & (idx >> np.uint64(b)) & np.uint64(1)).astype(bool)
                if sub[0] == "CCZ":
                    phi = np.where(on & ((idx >> np.uint64(t)) & np.uint64(1)).astype(bool), -phi, phi)
                else:
                    phi = phi[np.where(on, idx ^ (np.uint64(1) << np.uint64(t)), idx)]
                continue
            g, tok = sub[0], sub
        if g in ("H", "S", "SDG", "X", "Y", "Z", "H_XY", "H_NXY"):
            q = int(tok[1])
            phi = apply_1q(phi, MATS[g], q, n)
            shadow = apply_1q(shadow, MATS[g], q, n)
        elif g in ("T", "TDG"):
            phi = apply_1q(phi, MATS[g], int(tok[1]), n)
        elif g == "CX":
            phi = apply_cx(phi, int(tok[1]), int(tok[2]), n)
            shadow = apply_cx(shadow, int(tok[1]), int(tok[2]), n)
        elif g == "CZ":
            phi = apply_cz(phi, int(tok[1]), int(tok[2]), n)
            shadow = apply_cz(shadow, int(tok[1]), int(tok[2]), n)
        elif g in ("CCZ", "CCX"):
            # diag(..., -1 on x_a = x_b = x_t = 1); CCX flips t there instead.
            # Non-Clifford: the shadow stays.
            a, b, t = int(tok[1]), int(tok[2]), int(tok[3])
            idx = np.arange(1 << n, dtype=np.uint64)
            on = ((idx >> np.uint64(a)) & (idx >> np.uint64(b)) & np.uint64(1)).astype(bool)
            if g == "CCZ":
                phi = np.where(on & ((idx >> np.uint64(t)) & np.uint64(1)).astype(bool), -phi, phi)
            else:
                phi = phi[np.where(on, idx ^ (np.uint64(1) << np.uint64(t)), idx)]
        elif g in ("CS", "CSDG", "CPHASE", "RZ", "DIAG"):
            # textbook diagonal matrices: CS = diag(1, 1, 1, i), CSDG its
            # inverse, CPHASE(t) = diag(1, 1, 1, e^{it}), RZ(t) = exp(-i t Z / 2)
            # = diag(e^{-it/2}, e^{it/2}); DIAG k q.. phases: entry x of the
            # qubits (bit j = qubit q_j) gets e^{i phase_x}.  Non-Clifford in
            # general: the shadow stays.
            if g == "DIAG":
                k = int(tok[1])
                qs = [int(t) for t in tok[2:2 + k]]
                ph = [float(t) for t in tok[2 + k:]]
            elif g == "RZ":
                qs, t = [int(tok[2])], float(tok[1])
                ph = [-t / 2, t / 2]
            elif g == "CPHASE":
                qs, ph = [int(tok[2]), int(tok[3])], [0.0, 0.0, 0.0, float(tok[1])]
            else:
                qs, ph = [int(tok[1]), int(tok[2])], [0.0, 0.0, 0.0, np.pi / 2 if g == "CS" else -np.pi / 2]
            idx = np.arange(1 << n, dtype=np.uint64)
            x = np.zeros(1 << n, dtype=np.int64)
            for j, q in enumerate(qs):
                x |= ((idx >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << j
            phi = phi * np.exp(1j * np.asarray(ph))[x]
        elif g in ("XIF", "YIF", "ZIF"):
            # classically controlled Pauli
            if record[int(tok[1])]:
                q = int(tok[2])
                phi = apply_1q(phi, MATS[g[0]], q, n)
                shadow = apply_1q(shadow, MATS[g[0]], q, n)
        elif g in ("M", "R", "MPP", "MX", "RX", "MR", "MRX"):
            if g == "MPP":
                x, z = mpp_pauli(tok[1])
            elif g in ("MX", "RX", "MRX"):
                x, z = 1 << int(tok[1]), 0
            else:
                x, z = 0, 1 << int(tok[1])
            Pphi = pauli_apply(phi, x, z, 0, n)
            p0 = float(np.real(0.5 * (1 + np.vdot(phi, Pphi))))
            u = (float(meas_words[slot]) + 0.5) / 2.0 ** 32
            m = 1 if u < p0 else -1
            p0s.append(p0)
            slot += 1
            prob = p0 if m == 1 else 1 - p0
            phi = 0.5 * (phi + m * Pphi) / np.sqrt(prob)
            Psh = pauli_apply(shadow, x, z, 0, n)
            ev = np.vdot(shadow, Psh)
            if abs(abs(ev) - 1) < 1e-9:
                pass                          # deterministic on |psi_S>: unchanged
            elif abs(ev) < 1e-9:
                shadow = np.sqrt(2) * 0.5 * (shadow + m * Psh)
            else:
                raise AssertionError("shadow is not a stabilizer state")
            bit = 0 if m == 1 else 1
            if g not in ("R", "RX"):
                record.append(bit)
            if bit and g in ("R", "MR", "RX", "MRX"):
                # back to the +1 eigenstate: X flips Z_q, Z flips X_q
                F = MATS["X"] if g in ("R", "MR") else MATS["Z"]
                phi = apply_1q(phi, F, int(tok[1]), n)
                shadow = apply_1q(shadow, F, int(tok[1]), n)
        elif g in ("DETECTOR", "OBSERVABLE", "TICK"):
            pass
        else:
            raise ValueError("dense checker does not model " + g)
    return phi, shadow, record, p0s


def reconstruct(tab_x, tab_z, tab_r, coeffs, shadow, n):
    """sum_alpha v_alpha d_alpha |psi_S> from an oracle tableau and map."""
    out = np.zeros(1 << n, dtype=complex)
    for alpha, v in coeffs.items():
        vec = shadow.copy()
        for k in range(n):
            if (alpha >> k) & 1:
                vec = pauli_apply(vec, int(tab_x[k]), int(tab_z[k]), 2 * int(tab_r[k]), n)
        out += v * vec
    return out


def check_tableau(tab_x, tab_z, tab_r, shadow, n, tol=1e-10):
    """Stabilizer rows (with signs) fix the shadow; the symplectic relations
    d_i s_j = (-1)^{delta_ij} s_j d_i hold; stabilizers and destabilizers commute
    among themselves."""
    def anti(i, j):
        return bin((int(tab_x[i]) & int(tab_z[j])) ^ (int(tab_z[i]) & int(tab_x[j]))).count("1") & 1
    for i in range(n):
        s = n + i
        v = pauli_apply(shadow, int(tab_x[s]), int(tab_z[s]), 2 * int(tab_r[s]), n)
        assert np.max(np.abs(v - shadow)) < tol, "stabilizer %d does not fix |psi_S>" % i
        for j in range(n):
            assert anti(i, n + j) == (1 if i == j else 0)
            assert anti(i, j) == 0
            assert anti(n + i, n + j) == 0
