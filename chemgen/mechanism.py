"""Seeded synthetic reaction mechanisms and the versioned ``.mech`` text format.

This module builds *inputs*: species, NASA-7 thermo coefficients and elementary
reversible reactions drawn from a seed, following the recipe for the synthetic
stand-ins of the paper's H2 (9 species) and CH4 (20 species) mechanisms
(paper Section 4.1 and 4.2 name the real mechanisms; they are not available, so
seeded synthetic ones of the stated sizes replace them).  It evaluates no
reaction rate, right-hand side or integrator step: those belong to the method,
which the oracle and the GPU library each implement on their own.

The format is plain text so that the oracle (C) and the library (C++) each
parse it with their own reader.  Floats are written with ``repr`` (shortest
round-trip form), so both readers recover the exact binary64 values.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Sequence, Tuple

import numpy as np

#: Universal gas constant, J/(mol K) (CODATA 2018, exact).
R_U = 8.31446261815324
#: Reference temperature of formation enthalpies and standard entropies, K.
T_REF = 298.15
#: Atomic weights (g/mol) of the synthetic elements E0..E3.
ATOMIC_WEIGHTS = (1.008, 12.011, 15.999, 14.007)
FORMAT_VERSION = 1
GENERATOR_TAG = "chemgen-1"


@dataclasses.dataclass
class Mechanism:
    """A mechanism as plain data (no rate arithmetic).

    ``counts[k, e]`` is the number of atoms of element e in species k.
    ``nasa[k]`` holds 17 numbers: T_lo, T_mid, T_hi, seven low-range and seven
    high-range NASA-7 coefficients (cp/R = a1 + a2 T + ... + a5 T^4,
    a6 = enthalpy constant, a7 = entropy constant).
    A reaction is ``(reactants, products, A, b, Ea)``: each side is a list of
    ``(species, coefficient)`` pairs, A is in cm-mol-s units, Ea in J/mol.
    """

    element_names: List[str]
    element_weights: List[float]
    species_names: List[str]
    counts: np.ndarray
    nasa: np.ndarray
    reactions: List[Tuple[List[Tuple[int, int]], List[Tuple[int, int]], float, float, float]]
    seed: int = -1
    attempt: int = 0
    generator: str = GENERATOR_TAG

    @property
    def K(self) -> int:
        return len(self.species_names)

    @property
    def R(self) -> int:
        return len(self.reactions)

    @property
    def E(self) -> int:
        return len(self.element_names)

    def molar_masses(self) -> np.ndarray:
        """Species molar masses in kg/mol (sum of atomic weights)."""
        return 1e-3 * (self.counts @ np.asarray(self.element_weights, dtype=np.float64))

    def to_text(self) -> str:
        lines = [f"CHEMMECH {FORMAT_VERSION}",
                 f"generator {self.generator} seed {self.seed} attempt {self.attempt}",
                 "units A cm-mol-s Ea J/mol W g/mol",
                 f"elements {self.E}"]
        for n, w in zip(self.element_names, self.element_weights):
            lines.append(f"{n} {float(w)!r}")
        lines.append(f"species {self.K}")
        for k in range(self.K):
            cnt = " ".join(str(int(c)) for c in self.counts[k])
            coef = " ".join(repr(float(v)) for v in self.nasa[k])
            lines.append(f"{self.species_names[k]} {cnt} {coef}")
        lines.append(f"reactions {self.R}")
        for i, (reac, prod, A, b, Ea) in enumerate(self.reactions):
            rs = " ".join(f"{k} {nu}" for k, nu in reac)
            ps = " ".join(f"{k} {nu}" for k, nu in prod)
            lines.append(f"R{i} {len(reac)} {rs} {len(prod)} {ps} {float(A)!r} {float(b)!r} {float(Ea)!r}")
        lines.append("end")
        return "\n".join(lines) + "\n"

    def write(self, path: str) -> str:
        text = self.to_text()
        with open(path, "w") as fh:
            fh.write(text)
        return path

    def sha256(self) -> str:
        return hashlib.sha256(self.to_text().encode()).hexdigest()


def read_mechanism(path: str) -> Mechanism:
    """Parse a ``.mech`` file back into plain data (used by generators and tests)."""
    with open(path) as fh:
        tok = fh.read().split()
    pos = 0

    def nxt():
        nonlocal pos
        pos += 1
        return tok[pos - 1]

    assert nxt() == "CHEMMECH" and int(nxt()) == FORMAT_VERSION
    assert nxt() == "generator"
    gen = nxt()
    assert nxt() == "seed"
    seed = int(nxt())
    assert nxt() == "attempt"
    attempt = int(nxt())
    assert nxt() == "units"
    for _ in range(6):
        nxt()
    assert nxt() == "elements"
    E = int(nxt())
    en, ew = [], []
    for _ in range(E):
        en.append(nxt())
        ew.append(float(nxt()))
    assert nxt() == "species"
    K = int(nxt())
    sn, counts, nasa = [], np.zeros((K, E), dtype=np.int64), np.zeros((K, 17))
    for k in range(K):
        sn.append(nxt())
        for e in range(E):
            counts[k, e] = int(nxt())
        for j in range(17):
            nasa[k, j] = float(nxt())
    assert nxt() == "reactions"
    R = int(nxt())
    reactions = []
    for _ in range(R):
        nxt()
        nr = int(nxt())
        reac = [(int(nxt()), int(nxt())) for _ in range(nr)]
        np_ = int(nxt())
        prod = [(int(nxt()), int(nxt())) for _ in range(np_)]
        A, b, Ea = float(nxt()), float(nxt()), float(nxt())
        reactions.append((reac, prod, A, b, Ea))
    assert nxt() == "end"
    return Mechanism(en, ew, sn, counts, nasa, reactions, seed, attempt, gen)


# ----------------------------------------------------------------------------
# NASA-7 coefficient construction (input building only)
# ----------------------------------------------------------------------------

CP_NODES_T = (300.0, 1000.0, 2000.0, 3000.0)
CP_BOUNDS = (20.0, 60.0)
T_LO, T_MID, T_HI = 200.0, 1000.0, 3500.0


def _fit_cp_quartic(cp_nodes: Sequence[float]) -> np.ndarray:
    """Coefficients a1..a5 of cp/R through the four nodes with zero slope at 3000 K.

    Solved in the scaled variable theta = T/1000 for conditioning, then mapped
    back to powers of T.
    """
    th = np.array(CP_NODES_T) / 1000.0
    M = np.zeros((5, 5))
    rhs = np.zeros(5)
    for r, (t, c) in enumerate(zip(th, cp_nodes)):
        M[r] = [t ** j for j in range(5)]
        rhs[r] = c / R_U
    M[4] = [0.0] + [j * th[-1] ** (j - 1) for j in range(1, 5)]
    bcoef = np.linalg.solve(M, rhs)
    return np.array([bcoef[j] / 1000.0 ** j for j in range(5)])


def _cp_on_grid(a: np.ndarray) -> np.ndarray:
    T = np.arange(T_LO, T_HI + 0.5, 1.0)
    th = T / 1000.0
    b = [a[j] * 1000.0 ** j for j in range(5)]
    return R_U * (b[0] + th * (b[1] + th * (b[2] + th * (b[3] + th * b[4]))))


def _draw_thermo(rng: np.random.Generator, dhf_range, s0_range, bond_enthalpy=0.0,
                 bond_entropy=0.0, atoms=1) -> np.ndarray:
    """One species' 17 NASA numbers: cp nodes rising in [20, 60] J/(mol K);
    formation enthalpy ``-bond_enthalpy*(atoms - 1)`` plus a uniform draw from
    ``dhf_range``; standard entropy ``bond_entropy*(atoms - 1)`` plus a uniform
    draw from ``s0_range`` (both at 298.15 K)."""
    lo, hi = CP_BOUNDS
    while True:
        c0 = rng.uniform(20.0, 40.0)
        c1 = rng.uniform(c0, hi)
        c2 = rng.uniform(c1, hi)
        c3 = rng.uniform(c2, hi)
        a = _fit_cp_quartic((c0, c1, c2, c3))
        cp = _cp_on_grid(a)
        if cp.min() >= lo and cp.max() <= hi:
            break
    dhf = rng.uniform(*dhf_range) - bond_enthalpy * (atoms - 1)
    s0 = rng.uniform(*s0_range) + bond_entropy * (atoms - 1)
    t = T_REF
    h_int = a[0] * t + a[1] * t ** 2 / 2 + a[2] * t ** 3 / 3 + a[3] * t ** 4 / 4 + a[4] * t ** 5 / 5
    s_int = a[0] * math.log(t) + a[1] * t + a[2] * t ** 2 / 2 + a[3] * t ** 3 / 3 + a[4] * t ** 4 / 4
    a6 = dhf / R_U - h_int
    a7 = s0 / R_U - s_int
    coeffs = [a[0], a[1], a[2], a[3], a[4], a6, a7]
    return np.array([T_LO, T_MID, T_HI] + coeffs + coeffs, dtype=np.float64), dhf


# ----------------------------------------------------------------------------
# Species and reaction draws
# ----------------------------------------------------------------------------

def _species_candidates(E: int) -> np.ndarray:
    grids = np.array(np.meshgrid(*[np.arange(3)] * E, indexing="ij")).reshape(E, -1).T
    grids = grids[grids.sum(axis=1) > 0]
    # deterministic order: by total atoms, then lexicographic
    order = np.lexsort(tuple(grids[:, e] for e in reversed(range(E))) + (grids.sum(axis=1),))
    return grids[order]


def reaction_candidates(counts: np.ndarray) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """All unordered pairs of distinct sides with equal element totals.

    A side is one species ``(k,)`` or a multiset of two species ``(k, l)`` with
    k <= l.  The list order is deterministic.
    """
    K = counts.shape[0]
    sides = [(k,) for k in range(K)] + [(k, l) for k in range(K) for l in range(k, K)]
    groups = {}
    for s in sides:
        tot = tuple(int(v) for v in sum(counts[k] for k in s))
        groups.setdefault(tot, []).append(s)
    cands = []
    for tot in sorted(groups):
        g = groups[tot]
        for i in range(len(g)):
            for j in range(i + 1, len(g)):
                cands.append((g[i], g[j]))
    return cands


def _side_terms(side: Tuple[int, ...]) -> List[Tuple[int, int]]:
    if len(side) == 2 and side[0] == side[1]:
        return [(side[0], 2)]
    return [(k, 1) for k in side]


def make_mechanism(seed: int, K: int, R: int, E: int, *,
                   logA_range=(6.0, 14.0), b_range=(-1.0, 1.0), Ea_range=(0.0, 200e3),
                   dhf_range=(-40e3, 40e3), s0_range=(125.0, 175.0),
                   bond_enthalpy: float = 500e3, bond_entropy: float = 40.0,
                   orient: str = "exothermic",
                   max_attempts: int = 100000) -> Mechanism:
    """Draw a seeded element-balanced mechanism of K species, R reversible reactions.

    Species are distinct non-zero element-count vectors with counts 0..2, drawn
    without replacement with weight 1/(total atoms)^2.  If the species set admits
    fewer than R element-balanced candidate reactions the species set is redrawn
    from the sub-seed ``seed*1000 + attempt``; the attempt number is recorded.

    Thermo follows a bond-counting model: a species of ``a`` atoms has formation
    enthalpy ``-bond_enthalpy*(a-1) + U(dhf_range)`` and standard entropy
    ``bond_entropy*(a-1) + U(s0_range)``, so that bond formation is exothermic and
    dissociation gains entropy, as in combustion chemistry.  Each reaction is
    written in its exothermic direction (``orient="exothermic"``); the Arrhenius
    triple belongs to that direction and the reverse rate follows from K_c.
    """
    cand_species = _species_candidates(E)
    w = 1.0 / cand_species.sum(axis=1).astype(np.float64) ** 2
    w = w / w.sum()
    for attempt in range(max_attempts):
        rng = np.random.default_rng(seed if attempt == 0 else seed * 1000 + attempt)
        idx = rng.choice(len(cand_species), size=K, replace=False, p=w)
        counts = cand_species[np.sort(idx)]
        cands = reaction_candidates(counts)
        if len(cands) < R:
            continue
        thermo = [_draw_thermo(rng, dhf_range, s0_range, bond_enthalpy, bond_entropy,
                               int(counts[k].sum()))
                  for k in range(K)]
        nasa = np.stack([t[0] for t in thermo])
        dhf = np.array([t[1] for t in thermo])
        pick = rng.choice(len(cands), size=R, replace=False)
        coin = rng.random(R) < 0.5
        logA = rng.uniform(*logA_range, size=R)
        bb = rng.uniform(*b_range, size=R)
        Ea = rng.uniform(*Ea_range, size=R)
        reactions = []
        for i in range(R):
            s1, s2 = cands[pick[i]]
            if orient == "exothermic":
                # forward = the direction whose standard reaction enthalpy at 298.15 K is <= 0
                flip = sum(dhf[k] for k in s2) > sum(dhf[k] for k in s1)
            else:
                flip = bool(coin[i])
            if flip:
                s1, s2 = s2, s1
            reactions.append((_side_terms(s1), _side_terms(s2), float(10.0 ** logA[i]),
                              float(bb[i]), float(Ea[i])))
        return Mechanism([f"E{e}" for e in range(E)], list(ATOMIC_WEIGHTS[:E]),
                         [f"S{k}" for k in range(K)], counts.astype(np.int64), nasa,
                         reactions, seed, attempt)
    raise RuntimeError(f"no species set with >= {R} candidate reactions in {max_attempts} attempts")


#: The two synthetic mechanisms of the workloads: 9 species / 21 reactions /
#: 3 elements (stand-in for the H2 case) and 35 / 200 / 4 (larger than the CH4 case).
MECH_SPECS = {"M9": dict(seed=1, K=9, R=21, E=3), "M35": dict(seed=2, K=35, R=200, E=4)}


def standard_mechanism(name: str) -> Mechanism:
    return make_mechanism(**MECH_SPECS[name])


def custom_mechanism(counts, nasa_coeffs, reactions, element_weights=None,
                     species_names=None) -> Mechanism:
    """Build a mechanism from explicit data (test cases such as A <-> B isomers).

    ``nasa_coeffs[k]`` is a 7-vector used for both temperature ranges.
    """
    counts = np.asarray(counts, dtype=np.int64)
    K, E = counts.shape
    ew = list(element_weights) if element_weights is not None else list(ATOMIC_WEIGHTS[:E])
    nasa = np.array([[T_LO, T_MID, T_HI] + list(map(float, c)) + list(map(float, c))
                     for c in nasa_coeffs], dtype=np.float64)
    names = species_names or [f"S{k}" for k in range(K)]
    return Mechanism([f"E{e}" for e in range(E)], ew, names, counts, nasa,
                     [(list(r), list(p), float(A), float(b), float(Ea)) for r, p, A, b, Ea in reactions],
                     seed=-1, attempt=0, generator="custom")


def nasa_for(cp_over_R: Sequence[float], dhf: float, s0: float) -> List[float]:
    """Seven NASA coefficients for a given cp/R quartic (a1..a5) whose enthalpy at
    298.15 K equals ``dhf`` (J/mol) and entropy equals ``s0`` (J/(mol K))."""
    a = list(map(float, cp_over_R)) + [0.0] * (5 - len(cp_over_R))
    t = T_REF
    h_int = a[0] * t + a[1] * t ** 2 / 2 + a[2] * t ** 3 / 3 + a[3] * t ** 4 / 4 + a[4] * t ** 5 / 5
    s_int = a[0] * math.log(t) + a[1] * t + a[2] * t ** 2 / 2 + a[3] * t ** 3 / 3 + a[4] * t ** 4 / 4
    return a + [dhf / R_U - h_int, s0 / R_U - s_int]
