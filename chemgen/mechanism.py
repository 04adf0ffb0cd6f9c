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
from typing import List, Optional, Sequence, Tuple

import numpy as np

#: Universal gas constant, J/(mol K) (CODATA 2018, exact).
R_U = 8.31446261815324
#: Reference temperature of formation enthalpies and standard entropies, K.
T_REF = 298.15
#: Atomic weights (g/mol) of the synthetic elements E0..E3.
ATOMIC_WEIGHTS = (1.008, 12.011, 15.999, 14.007)
FORMAT_VERSION = 1
#: Version written when a reaction is not elementary-reversible (three-body,
#: fall-off, irreversible); version 1 files stay byte-identical.
FORMAT_VERSION_KINETICS = 2
GENERATOR_TAG = "chemgen-1"

#: Pressure-dependence kinds of the version 2 format.
KINDS = ("elem", "third", "lind", "troe3", "troe4")


@dataclasses.dataclass
class RxnKinetics:
    """What a reaction has beyond a reversible mass-action Arrhenius rate.

    ``kind``: "elem" (none), "third" (rate times the third-body concentration
    [M]), "lind" / "troe3" / "troe4" (fall-off between the low-pressure rate
    ``low`` = (A0, b0, Ea0) times [M] and the reaction's own Arrhenius triple
    as the high-pressure limit; Lindemann, or Troe broadening with
    ``troe`` = (a, T3, T1) or (a, T3, T1, T2)).  [M] = ``default_eff`` times
    the total concentration plus ``(eff - default_eff) C_k`` for every listed
    ``(k, eff)``.  ``reversible=False``: no reverse rate.  A0 is in cm-mol-s
    units of one order above A; Ea0 in J/mol.
    """

    kind: str = "elem"
    reversible: bool = True
    default_eff: float = 1.0
    effs: List[Tuple[int, float]] = dataclasses.field(default_factory=list)
    low: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    troe: Tuple[float, ...] = ()

    def is_plain(self) -> bool:
        return self.kind == "elem" and self.reversible


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
    #: per reaction, None for an elementary reversible one (None: all are)
    kinetics: Optional[List[Optional[RxnKinetics]]] = None

    def kin(self, i: int) -> RxnKinetics:
        if self.kinetics is None or self.kinetics[i] is None:
            return RxnKinetics()
        return self.kinetics[i]

    def plain(self) -> bool:
        return all(self.kin(i).is_plain() for i in range(self.R))

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
        v2 = not self.plain()
        lines = [f"CHEMMECH {FORMAT_VERSION_KINETICS if v2 else FORMAT_VERSION}",
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
            line = f"R{i} {len(reac)} {rs} {len(prod)} {ps} {float(A)!r} {float(b)!r} {float(Ea)!r}"
            if v2:
                line += " " + _kinetics_text(self.kin(i))
            lines.append(line)
        lines.append("end")
        return "\n".join(lines) + "\n"

    def write(self, path: str) -> str:
        text = self.to_text()
        with open(path, "w") as fh:
            fh.write(text)
        return path

    def sha256(self) -> str:
        return hashlib.sha256(self.to_text().encode()).hexdigest()


def _kinetics_text(x: RxnKinetics) -> str:
    """Version 2 tail of a reaction line: reversibility flag, kind, then for
    pressure-dependent kinds the low-pressure triple (fall-off), the Troe
    parameters, the default efficiency and the listed efficiencies."""
    out = [str(int(x.reversible)), x.kind]
    if x.kind in ("lind", "troe3", "troe4"):
        out += [repr(float(v)) for v in x.low]
    if x.kind == "troe3":
        out += [repr(float(v)) for v in x.troe[:3]]
    if x.kind == "troe4":
        out += [repr(float(v)) for v in x.troe[:4]]
    if x.kind != "elem":
        out += [repr(float(x.default_eff)), str(len(x.effs))]
        for k, e in x.effs:
            out += [str(int(k)), repr(float(e))]
    return " ".join(out)


def read_mechanism(path: str) -> Mechanism:
    """Parse a ``.mech`` file back into plain data (used by generators and tests)."""
    with open(path) as fh:
        tok = fh.read().split()
    pos = 0

    def nxt():
        nonlocal pos
        pos += 1
        return tok[pos - 1]

    assert nxt() == "CHEMMECH"
    version = int(nxt())
    assert version in (FORMAT_VERSION, FORMAT_VERSION_KINETICS)
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
    reactions, kinetics = [], []
    for _ in range(R):
        nxt()
        nr = int(nxt())
        reac = [(int(nxt()), int(nxt())) for _ in range(nr)]
        np_ = int(nxt())
        prod = [(int(nxt()), int(nxt())) for _ in range(np_)]
        A, b, Ea = float(nxt()), float(nxt()), float(nxt())
        reactions.append((reac, prod, A, b, Ea))
        x = None
        if version == FORMAT_VERSION_KINETICS:
            x = RxnKinetics(reversible=bool(int(nxt())), kind=nxt())
            assert x.kind in KINDS
            if x.kind in ("lind", "troe3", "troe4"):
                x.low = (float(nxt()), float(nxt()), float(nxt()))
            if x.kind in ("troe3", "troe4"):
                x.troe = tuple(float(nxt()) for _ in range(3 if x.kind == "troe3" else 4))
            if x.kind != "elem":
                x.default_eff = float(nxt())
                x.effs = [(int(nxt()), float(nxt())) for _ in range(int(nxt()))]
        kinetics.append(x)
    assert nxt() == "end"
    return Mechanism(en, ew, sn, counts, nasa, reactions, seed, attempt, gen,
                     kinetics if any(x is not None for x in kinetics) else None)


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


def _second_range(rng: np.random.Generator, nasa_row: np.ndarray, scale: float = 0.05) -> np.ndarray:
    """Give a species a high-temperature NASA-7 range of its own.

    The high range is the low one plus a cp/R correction
    e1 (T - Tmid) + e2 (T - Tmid)^2 that vanishes at Tmid, with the enthalpy
    and entropy constants chosen so that cp, H and S are continuous at Tmid
    (as fitted NASA-7 data are); cp/R stays within ``scale`` times its own
    range over [Tmid, Thi]."""
    out = nasa_row.copy()
    tm, th = nasa_row[1], nasa_row[2]
    span = th - tm
    e1 = rng.uniform(-1.0, 1.0) * scale * 4.0 / span
    e2 = rng.uniform(-1.0, 1.0) * scale * 4.0 / span ** 2
    d = np.zeros(7)
    d[0] = -e1 * tm + e2 * tm * tm
    d[1] = e1 - 2.0 * e2 * tm
    d[2] = e2
    d[5] = -(d[0] * tm + d[1] * tm ** 2 / 2.0 + d[2] * tm ** 3 / 3.0)
    d[6] = -(d[0] * math.log(tm) + d[1] * tm + d[2] * tm ** 2 / 2.0)
    out[10:17] = nasa_row[3:10] + d
    return out


def make_real_like_mechanism(seed: int, K: int, R: int, E: int, *, n_third: int, n_lind: int,
                             n_troe: int, n_dup: int, n_irrev: int) -> Mechanism:
    """A seeded mechanism with the features of real combustion mechanisms.

    Starts from ``make_mechanism`` (R - n_dup elementary reactions) and then:
    every species gets a high-temperature NASA range of its own
    (``_second_range``); n_third recombination / dissociation reactions (one
    species on one side, two on the other) become three-body reactions and
    n_lind + n_troe more become fall-off reactions (Lindemann, then Troe with
    three and four parameters alternately), each with a few listed collision
    efficiencies (one of them 0) and, for one reaction, a single bath species
    (default efficiency 0); n_dup reactions get a duplicate with their own
    Arrhenius triple; n_irrev elementary reactions become irreversible.
    Three-body and low-pressure pre-exponentials are drawn 10^4..10^6.5 times
    the bimolecular one, so that at 1 atm and flame temperatures the fall-off
    reactions sit inside their fall-off range (reduced pressure about 0.1-100).
    """
    base = make_mechanism(seed, K, R - n_dup, E)
    rng = np.random.default_rng(seed * 7919 + 17)
    nasa = np.stack([_second_range(rng, base.nasa[k]) for k in range(K)])
    reactions = list(base.reactions)
    kin: List[Optional[RxnKinetics]] = [None] * len(reactions)
    uni = [i for i, (r, p, *_) in enumerate(reactions)
           if sum(nu for _, nu in r) + sum(nu for _, nu in p) == 3]
    n_pd = n_third + n_lind + n_troe
    if len(uni) < n_pd:
        raise ValueError(f"only {len(uni)} reactions with one and two molecules on their sides")
    pick = [uni[j] for j in rng.choice(len(uni), size=n_pd, replace=False)]
    for j, i in enumerate(pick):
        reac, prod, A, b, Ea = reactions[i]
        neff = int(rng.integers(2, 4))
        ks = rng.choice(K, size=neff, replace=False)
        effs = [(int(k), 0.0 if t == 0 else float(np.round(rng.uniform(0.3, 12.0), 2)))
                for t, k in enumerate(sorted(ks))]
        x = RxnKinetics(effs=effs)
        if j == 0:
            x.default_eff = 0.0
            x.effs = [(int(ks[0]), 1.0)]
        if j < n_third:
            x.kind = "third"
            reactions[i] = (reac, prod, A * 10.0 ** rng.uniform(4.0, 6.5), b, Ea)
        else:
            x.low = (A * 10.0 ** rng.uniform(4.0, 6.5), float(rng.uniform(-2.0, 0.0)),
                     float(rng.uniform(0.0, 0.5)) * Ea)
            if j < n_third + n_lind:
                x.kind = "lind"
            else:
                t = j - n_third - n_lind
                x.kind = "troe3" if t % 2 == 0 else "troe4"
                troe = (float(np.round(rng.uniform(0.3, 0.9), 3)), float(np.round(rng.uniform(50.0, 400.0), 1)),
                        float(np.round(rng.uniform(800.0, 3000.0), 1)))
                if x.kind == "troe4":
                    troe += (float(np.round(rng.uniform(3000.0, 8000.0), 1)),)
                x.troe = troe
        kin[i] = x
    rest = [i for i in range(len(reactions)) if kin[i] is None]
    for i in rng.choice(rest, size=n_irrev, replace=False):
        kin[int(i)] = RxnKinetics(reversible=False)
    for i in rng.choice(len(reactions), size=n_dup, replace=False):
        reac, prod, A, b, Ea = reactions[int(i)]
        reactions.append((reac, prod, float(A * 10.0 ** rng.uniform(-1.5, 0.5)), float(rng.uniform(-1.0, 1.0)),
                          float(rng.uniform(0.0, 200e3))))
        src = kin[int(i)]
        kin.append(dataclasses.replace(src, effs=list(src.effs)) if src is not None else None)
    return Mechanism(base.element_names, base.element_weights, base.species_names, base.counts, nasa,
                     reactions, seed, base.attempt, "chemgen-2", kin)


#: The synthetic mechanisms of the workloads: 9 species / 21 reactions /
#: 3 elements (stand-in for the H2 case) and 35 / 200 / 4 (larger than the CH4
#: case), elementary reversible reactions with one NASA range; and two with the
#: features of real mechanisms at the sizes of the paper's H2 and CH4 cases
#: (9 species / 12 reactions, 20 species / 85 reactions): three-body and
#: fall-off reactions, duplicates, irreversible reactions, two NASA ranges.
MECH_SPECS = {"M9": dict(seed=1, K=9, R=21, E=3), "M35": dict(seed=2, K=35, R=200, E=4)}
REAL_LIKE_SPECS = {
    "H2R": dict(seed=3, K=9, R=12, E=3, n_third=2, n_lind=1, n_troe=2, n_dup=1, n_irrev=1),
    "CH4R": dict(seed=4, K=20, R=85, E=4, n_third=8, n_lind=3, n_troe=4, n_dup=4, n_irrev=3),
}


def standard_mechanism(name: str) -> Mechanism:
    if name in REAL_LIKE_SPECS:
        return make_real_like_mechanism(**REAL_LIKE_SPECS[name])
    return make_mechanism(**MECH_SPECS[name])


def custom_mechanism(counts, nasa_coeffs, reactions, element_weights=None,
                     species_names=None, kinetics=None) -> Mechanism:
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
                     seed=-1, attempt=0, generator="custom", kinetics=kinetics)


def nasa_for(cp_over_R: Sequence[float], dhf: float, s0: float) -> List[float]:
    """Seven NASA coefficients for a given cp/R quartic (a1..a5) whose enthalpy at
    298.15 K equals ``dhf`` (J/mol) and entropy equals ``s0`` (J/(mol K))."""
    a = list(map(float, cp_over_R)) + [0.0] * (5 - len(cp_over_R))
    t = T_REF
    h_int = a[0] * t + a[1] * t ** 2 / 2 + a[2] * t ** 3 / 3 + a[3] * t ** 4 / 4 + a[4] * t ** 5 / 5
    s_int = a[0] * math.log(t) + a[1] * t + a[2] * t ** 2 / 2 + a[3] * t ** 3 / 3 + a[4] * t ** 4 / 4
    return a + [dhf / R_U - h_int, s0 / R_U - s_int]
