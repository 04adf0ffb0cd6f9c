"""CHEMKIN-format mechanisms to and from the ``.mech`` format.

Reads the ELEMENTS, SPECIES, THERMO (NASA-7 records; or a separate thermo
file) and REACTIONS sections of a CHEMKIN-II style mechanism and builds a
:class:`chemgen.mechanism.Mechanism`, so that a user's mechanism (the paper's
H2 and CH4 cases, Sections 4.1 and 4.2, are such files) can be converted once
and then read by the library and the oracle.  Conversion only: units are
brought to cm-mol-s and J/mol, and nothing of the kinetics is evaluated.

Supported reaction syntax: ``<=>``, ``=`` (reversible) and ``=>``
(irreversible); integer stoichiometric prefixes (``2OH``); ``+M`` third-body
reactions; ``(+M)`` and ``(+species)`` fall-off with ``LOW/.../`` and an
optional ``TROE/a T3 T1 [T2]/`` line; collision efficiencies
(``SP/value/``); ``DUPLICATE``/``DUP``; a species present on both sides of a
reaction with three molecules on a side (``H+O2+H2O<=>HO2+H2O``), which is
a three-body reaction with that species as the only collider; the units
keywords of the REACTIONS line (CAL/MOLE, KCAL/MOLE, JOULES/MOLE,
KJOULES/MOLE, KELVINS; MOLES).  Anything else (REV, PLOG, CHEB, SRI, FORD,
MOLECULES, more than two molecules on a side) is rejected with an error.
"""
from __future__ import annotations

import re
from typing import Dict, List, Optional, Tuple

import numpy as np

from .mechanism import R_U, Mechanism, RxnKinetics

#: Standard atomic weights (g/mol) of the elements the converter knows.
ATOMIC_WEIGHT = {"H": 1.008, "HE": 4.0026, "C": 12.011, "N": 14.007, "O": 15.999, "AR": 39.948,
                 "NE": 20.180, "F": 18.998, "CL": 35.45, "S": 32.06}

_EA_FACTOR = {"CAL/MOLE": 4.184, "KCAL/MOLE": 4184.0, "JOULES/MOLE": 1.0, "KJOULES/MOLE": 1000.0,
              "KELVINS": R_U}


class ChemkinError(ValueError):
    pass


def _strip(line: str) -> str:
    return line.split("!", 1)[0].rstrip()


def _sections(text: str) -> Dict[str, Tuple[List[str], List[str]]]:
    """Per section (ELEM/ELEMENTS, SPEC/SPECIES, THERMO, REAC/REACTIONS): the
    words after the keyword on its own line (up to an END there) and the
    following lines up to the END line."""
    out: Dict[str, Tuple[List[str], List[str]]] = {}
    cur = None
    for raw in text.splitlines():
        line = _strip(raw)
        words = line.split()
        key = {"ELEM": "ELEMENTS", "ELEMENTS": "ELEMENTS", "SPEC": "SPECIES", "SPECIES": "SPECIES",
               "THERMO": "THERMO", "REAC": "REACTIONS", "REACTIONS": "REACTIONS"}.get(
            words[0].upper() if words else "")
        if key:
            rest = words[1:]
            closed = any(w.upper() == "END" for w in rest)
            if closed:
                rest = rest[:[w.upper() for w in rest].index("END")]
            out[key] = (rest, [])
            cur = None if closed else key
            continue
        if [w.upper() for w in words] == ["END"]:
            cur = None
            continue
        if cur and line.strip():
            if words[-1].upper() == "END" and cur in ("ELEMENTS", "SPECIES"):
                out[cur][1].append(" ".join(words[:-1]))
                cur = None
                continue
            out[cur][1].append(line)
    return out


def _words(sec: Tuple[List[str], List[str]]) -> List[str]:
    return sec[0] + " ".join(sec[1]).split()


def _parse_thermo(lines: List[str], want: List[str]) -> Dict[str, Tuple[Dict[str, int], np.ndarray]]:
    """NASA-7 records (four 80-column lines each) of the wanted species:
    element counts and [Tlo, Tmid, Thi, low 7, high 7]."""
    body = [ln for ln in lines if ln.strip()]
    tdef = (300.0, 1000.0, 5000.0)
    i = 0
    if body and re.fullmatch(r"\s*[-+0-9.eEdD]+\s+[-+0-9.eEdD]+\s+[-+0-9.eEdD]+\s*", body[0]):
        tdef = tuple(float(v) for v in body[0].split())
        i = 1
    out = {}
    wanted = {s.upper() for s in want}
    while i + 3 < len(body) + 0 and i < len(body):
        l1 = body[i].ljust(80)
        if i + 3 >= len(body):
            break
        name = l1[:18].split()[0] if l1[:18].split() else ""
        comp: Dict[str, int] = {}
        for j in range(4):
            el, cnt = l1[24 + 5 * j: 26 + 5 * j].strip(), l1[26 + 5 * j: 29 + 5 * j].strip()
            if el and cnt and el != "0":
                n = int(float(cnt))
                if n:
                    comp[el.upper()] = comp.get(el.upper(), 0) + n
        el5, cnt5 = l1[73:75].strip(), l1[75:78].strip()
        if el5 and cnt5 and el5 != "0" and int(float(cnt5)):
            comp[el5.upper()] = comp.get(el5.upper(), 0) + int(float(cnt5))
        try:
            tlo = float(l1[45:55]) if l1[45:55].strip() else tdef[0]
            thi = float(l1[55:65]) if l1[55:65].strip() else tdef[2]
            tmid = float(l1[65:73]) if l1[65:73].strip() else tdef[1]
            coef = []
            for k in range(1, 4):
                row = body[i + k].ljust(80)
                for j in range(5):
                    f = row[15 * j: 15 * j + 15].strip().replace("D", "E").replace("d", "e")
                    if f:
                        coef.append(float(f))
        except ValueError as e:
            raise ChemkinError(f"bad thermo record of {name}: {e}")
        if len(coef) < 14:
            raise ChemkinError(f"thermo record of {name} has {len(coef)} coefficients")
        if name.upper() in wanted and name.upper() not in out:
            high, low = coef[0:7], coef[7:14]
            out[name.upper()] = (comp, np.array([tlo, tmid, thi] + low + high, dtype=np.float64))
        i += 4
    return out


_SLASH = re.compile(r"([A-Za-z0-9_()*,\-+#\[\]]+)\s*/\s*([^/]*)/")


def _side(text: str, index: Dict[str, int]) -> Tuple[List[Tuple[int, int]], Optional[str], bool]:
    """Species of one side, the fall-off collider ('M' or a species, None)
    and whether a '+M' third body is present."""
    collider = None
    m = re.search(r"\(\+\s*([A-Za-z0-9_*\-,\[\]#]+)\s*\)", text)
    if m:
        collider = m.group(1).upper()
        text = text[:m.start()] + text[m.end():]
    terms = [t.strip() for t in re.split(r"\+(?![^(]*\))", text) if t.strip()]
    third = False
    out: Dict[int, int] = {}
    for t in terms:
        if t.upper() == "M":
            third = True
            continue
        mm = re.fullmatch(r"(\d*)\s*(.+)", t)
        nu = int(mm.group(1)) if mm.group(1) else 1
        sp = mm.group(2).upper()
        if sp not in index:
            raise ChemkinError(f"unknown species {sp} in '{text}'")
        out[index[sp]] = out.get(index[sp], 0) + nu
    return sorted(out.items()), collider, third


def parse_chemkin(mech_text: str, thermo_text: Optional[str] = None, name: str = "chemkin") -> Mechanism:
    """Build a Mechanism from CHEMKIN text (thermo in the mechanism's THERMO
    section, or in thermo_text)."""
    sec = _sections(mech_text)
    elements, weights = [], {}
    for w in _words(sec.get("ELEMENTS", ([], []))):
        mm = re.fullmatch(r"([A-Za-z0-9]+)(?:/\s*([-+0-9.eEdD]+)\s*/)?", w)
        if not mm:
            raise ChemkinError(f"bad element entry {w}")
        e = mm.group(1).upper()
        elements.append(e)
        if mm.group(2):
            weights[e] = float(mm.group(2).replace("D", "E").replace("d", "e"))
        elif e in ATOMIC_WEIGHT:
            weights[e] = ATOMIC_WEIGHT[e]
        else:
            raise ChemkinError(f"no atomic weight for element {e}")
    if not elements:
        raise ChemkinError("no ELEMENTS section")
    species = [s.upper() for s in _words(sec.get("SPECIES", ([], [])))]
    if not species:
        raise ChemkinError("no SPECIES section")
    index = {s: k for k, s in enumerate(species)}
    tlines = sec.get("THERMO", ([], []))[1]
    if thermo_text is not None:
        tlines = _sections(thermo_text if thermo_text.lstrip().upper().startswith("THERMO")
                           else "THERMO\n" + thermo_text).get("THERMO", ([], []))[1]
    thermo = _parse_thermo(tlines, species)
    missing = [s for s in species if s not in thermo]
    if missing:
        raise ChemkinError(f"no thermo data for {missing}")
    counts = np.zeros((len(species), len(elements)), dtype=np.int64)
    for s, k in index.items():
        for el, n in thermo[s][0].items():
            if el not in elements:
                raise ChemkinError(f"species {s} has element {el} that ELEMENTS does not list")
            counts[k, elements.index(el)] = n
    nasa = np.stack([thermo[s][1] for s in species])

    header, rlines = sec.get("REACTIONS", ([], []))
    header = [w.upper() for w in header]
    ea_factor = 4.184
    for w in header:
        if w in _EA_FACTOR:
            ea_factor = _EA_FACTOR[w]
        elif w == "MOLECULES":
            raise ChemkinError("A in molecules units is not supported")
        elif w not in ("MOLES",):
            raise ChemkinError(f"unknown units keyword {w}")
    reactions, kinetics = [], []
    cur = None
    for line in rlines:
        s = line.strip()
        up = s.upper()
        if "=" in s and not up.startswith(("LOW", "TROE", "REV", "PLOG", "CHEB", "SRI", "FORD", "DUP")):
            toks = s.split()
            if len(toks) < 4:
                raise ChemkinError(f"bad reaction line '{s}'")
            eq = "".join(toks[:-3])
            A, b, Ea = (float(t.replace("D", "E").replace("d", "e")) for t in toks[-3:])
            if "<=>" in eq:
                lhs, rhs, rev = *eq.split("<=>"), True
            elif "=>" in eq:
                lhs, rhs, rev = *eq.split("=>"), False
            else:
                lhs, rhs, rev = *eq.split("="), True
            reac, cl, third_l = _side(lhs, index)
            prod, cr, third_r = _side(rhs, index)
            if cl != cr or third_l != third_r:
                raise ChemkinError(f"third body differs between the sides of '{s}'")
            x = RxnKinetics(reversible=rev)
            if third_l:
                x.kind = "third"
            elif cl is not None:
                x.kind = "lind"
                if cl != "M":
                    if cl not in index:
                        raise ChemkinError(f"unknown collider {cl}")
                    x.default_eff, x.effs = 0.0, [(index[cl], 1.0)]
            # a species on both sides of a three-molecule side: the only collider
            if x.kind == "elem" and (sum(n for _, n in reac) > 2 or sum(n for _, n in prod) > 2):
                common = sorted(set(k for k, _ in reac) & set(k for k, _ in prod))
                if not common:
                    raise ChemkinError(f"more than two molecules on a side of '{s}'")
                c = common[0]
                reac = [(k, n - (k == c)) for k, n in reac if n - (k == c) > 0]
                prod = [(k, n - (k == c)) for k, n in prod if n - (k == c) > 0]
                x.kind, x.default_eff, x.effs = "third", 0.0, [(c, 1.0)]
            if sum(n for _, n in reac) > 2 or sum(n for _, n in prod) > 2:
                raise ChemkinError(f"more than two molecules on a side of '{s}'")
            reactions.append((reac, prod, A, b, Ea * ea_factor))
            kinetics.append(x)
            cur = x
            continue
        if cur is None:
            raise ChemkinError(f"auxiliary line before any reaction: '{s}'")
        if up.startswith("DUP"):
            continue
        for key, val in _SLASH.findall(s):
            k = key.upper()
            vals = [float(v.replace("D", "E").replace("d", "e")) for v in val.split()]
            if k == "LOW":
                if cur.kind not in ("lind", "troe3", "troe4") or len(vals) != 3:
                    raise ChemkinError(f"LOW on a reaction that is not a fall-off: '{s}'")
                cur.low = (vals[0], vals[1], vals[2] * ea_factor)
            elif k == "TROE":
                if cur.kind not in ("lind", "troe3", "troe4") or len(vals) not in (3, 4):
                    raise ChemkinError(f"bad TROE line '{s}'")
                cur.kind = "troe3" if len(vals) == 3 else "troe4"
                cur.troe = tuple(vals)
            elif k in ("REV", "PLOG", "CHEB", "SRI", "FORD", "RORD", "HIGH", "LT", "RLT", "TDEP", "EXCI", "UNITS"):
                raise ChemkinError(f"{k} is not supported")
            elif k in index:
                if cur.kind == "elem":
                    raise ChemkinError(f"efficiency on a reaction without a third body: '{s}'")
                if len(vals) != 1:
                    raise ChemkinError(f"bad efficiency '{s}'")
                cur.effs = [(kk, v) for kk, v in cur.effs if kk != index[k]] + [(index[k], vals[0])]
            else:
                raise ChemkinError(f"unknown keyword or species {k}")
    for x in kinetics:
        if x.kind in ("lind", "troe3", "troe4") and x.low == (0.0, 0.0, 0.0):
            raise ChemkinError("fall-off reaction without LOW")
        x.effs = sorted(x.effs)
    return Mechanism(elements, [weights[e] for e in elements], species, counts, nasa, reactions,
                     seed=-1, attempt=0, generator=name, kinetics=kinetics if kinetics else None)


def _fmt(v: float) -> str:
    return f"{v:15.8E}"


def to_chemkin(m: Mechanism) -> str:
    """CHEMKIN text of a Mechanism (elements named as in it, with their
    weights; thermo in the standard four-line records; A in cm-mol-s, Ea in
    J/mol: JOULES/MOLE)."""
    L = ["ELEMENTS", " ".join(f"{n}/{float(w)!r}/" for n, w in zip(m.element_names, m.element_weights)), "END",
         "SPECIES", " ".join(m.species_names), "END",
         "THERMO ALL", "   200.000  1000.000  3500.000"]
    for k, s in enumerate(m.species_names):
        comp = "".join(f"{m.element_names[e]:<2}{int(m.counts[k, e]):>3}" for e in range(m.E) if m.counts[k, e])
        comp = comp[:20].ljust(20)
        tlo, tmid, thi = m.nasa[k, :3]
        L.append(f"{s:<18}      {comp}G{tlo:10.3f}{thi:10.3f}{tmid:8.2f}      1")
        c = list(m.nasa[k, 10:17]) + list(m.nasa[k, 3:10])
        L.append("".join(_fmt(v) for v in c[0:5]) + "    2")
        L.append("".join(_fmt(v) for v in c[5:10]) + "    3")
        L.append("".join(_fmt(v) for v in c[10:14]) + "                   4")
    L += ["END", "REACTIONS JOULES/MOLE MOLES"]

    def side(terms, coll, third):
        s = "+".join((f"{nu}" if nu > 1 else "") + m.species_names[k] for k, nu in terms)
        return s + ("+M" if third else "") + (f"(+{coll})" if coll else "")

    keys = [(tuple(r), tuple(p)) for r, p, *_ in m.reactions]
    for i, (r, p, A, b, Ea) in enumerate(m.reactions):
        x = m.kin(i)
        third = x.kind == "third"
        coll = None
        if x.kind in ("lind", "troe3", "troe4"):
            coll = "M"
            if x.default_eff == 0.0 and len(x.effs) == 1 and x.effs[0][1] == 1.0:
                coll = m.species_names[x.effs[0][0]]
        arrow = "<=>" if x.reversible else "=>"
        L.append(f"{side(r, coll, third)}{arrow}{side(p, coll, third)}   {A!r} {b!r} {Ea!r}")
        if x.kind in ("lind", "troe3", "troe4"):
            L.append(f"    LOW/ {x.low[0]!r} {x.low[1]!r} {x.low[2]!r} /")
        if x.kind in ("troe3", "troe4"):
            L.append("    TROE/ " + " ".join(repr(float(v)) for v in x.troe) + " /")
        if x.kind != "elem" and coll in (None, "M"):
            if x.default_eff != 1.0:
                if not (third and x.default_eff == 0.0 and len(x.effs) == 1):
                    raise ChemkinError("a default efficiency other than 1 has no CHEMKIN form")
            effs = [(k, e) for k, e in x.effs if e != 1.0 or x.default_eff != 1.0]
            if third and x.default_eff == 0.0:
                # sole collider: written as the species on both sides
                k = x.effs[0][0]
                L[-1] = (f"{side(r, None, False)}+{m.species_names[k]}{arrow}{side(p, None, False)}+"
                         f"{m.species_names[k]}   {A!r} {b!r} {Ea!r}")
                effs = []
            if effs:
                L.append("    " + " ".join(f"{m.species_names[k]}/{e!r}/" for k, e in effs))
        if keys.count(keys[i]) > 1:
            L.append("    DUPLICATE")
    L.append("END")
    return "\n".join(L) + "\n"
