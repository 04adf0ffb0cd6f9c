"""The CHEMKIN converter (chemgen.chemkin): round trip of the real-mechanism
stand-ins through CHEMKIN text, the reaction syntax it accepts (checked value
by value on a hand-written reaction section over made-up species), and the
forms it rejects."""
import math

import numpy as np
import pytest

from chemgen.chemkin import ChemkinError, parse_chemkin, to_chemkin
from chemgen.mechanism import custom_mechanism, standard_mechanism


@pytest.mark.parametrize("name", ["H2R", "CH4R", "M9"])
def test_round_trip(name):
    m = standard_mechanism(name)
    b = parse_chemkin(to_chemkin(m))
    assert b.species_names == m.species_names and b.element_names == m.element_names
    assert np.array_equal(b.counts, m.counts) and b.element_weights == m.element_weights
    # thermo records carry 9 significant digits (E15.8)
    assert np.allclose(b.nasa, m.nasa, rtol=1e-8, atol=0)
    assert b.reactions == m.reactions
    for i in range(m.R):
        x, y = m.kin(i), b.kin(i)
        assert (x.kind, x.reversible, x.default_eff, x.effs, x.low, tuple(x.troe)) == \
               (y.kind, y.reversible, y.default_eff, y.effs, y.low, tuple(y.troe))


def _thermo_block():
    """Thermo records of six made-up species in two elements, written by the
    converter's own writer (fixed columns are tedious to type)."""
    counts = [[1, 0], [0, 1], [1, 1], [2, 0], [0, 2], [2, 1]]
    coeffs = [[3.0 + 0.1 * k, 1e-3, -1e-7, 0.0, 0.0, -1000.0 * k, 2.0 + k] for k in range(6)]
    m = custom_mechanism(counts, coeffs, [([(0, 1), (1, 1)], [(2, 1)], 1.0, 0.0, 0.0)],
                         element_weights=[1.008, 15.999], species_names=["A", "B", "AB", "A2", "B2", "A2B"])
    m.element_names = ["H", "O"]
    text = to_chemkin(m)
    return text[text.index("THERMO"):text.index("REACTIONS")]


REACTIONS = """
REACTIONS KCAL/MOLE
! comment line
A+B=AB               1.0E13  0.5  2.0     ! reversible, '='
2A=>A2               3.0E12  0.0  0.0     ! irreversible
A+B+M<=>AB+M         5.0E16 -1.0  0.0
   A2/2.5/ B2/0.0/
A+AB(+M)<=>A2B(+M)   2.0E12  0.2  1.0
   LOW / 4.0E17 -1.5 0.5 /
A+A(+B2)<=>A2(+B2)   7.0E11  0.0  0.0
   LOW / 1.0E16 0.0 0.0 /
   TROE / 0.6 100.0 2000.0 5000.0 /
A+B2+A2B<=>AB+B+A2B  6.0E15  0.0  0.0
B+B<=>B2             1.0E12  0.0  0.0
   DUPLICATE
B+B<=>B2             2.0E10  1.0  0.0
   DUP
END
"""


def test_reaction_syntax():
    text = "ELEMENTS H O END\nSPECIES A B AB A2 B2 A2B END\n" + _thermo_block() + REACTIONS
    m = parse_chemkin(text)
    assert m.element_weights == [1.008, 15.999]
    sp = {s: k for k, s in enumerate(m.species_names)}
    A, B, AB, A2, B2, A2B = (sp[s] for s in ("A", "B", "AB", "A2", "B2", "A2B"))
    r = m.reactions
    assert len(r) == 8
    # Ea from kcal/mol to J/mol, A unchanged
    assert r[0] == ([(A, 1), (B, 1)], [(AB, 1)], 1.0e13, 0.5, 2.0 * 4184.0)
    assert m.kin(0).kind == "elem" and m.kin(0).reversible
    assert r[1][:2] == ([(A, 2)], [(A2, 1)]) and not m.kin(1).reversible
    x = m.kin(2)
    assert x.kind == "third" and x.default_eff == 1.0 and x.effs == [(A2, 2.5), (B2, 0.0)]
    x = m.kin(3)
    assert x.kind == "lind" and x.low == (4.0e17, -1.5, 0.5 * 4184.0) and x.effs == []
    x = m.kin(4)
    assert x.kind == "troe4" and x.troe == (0.6, 100.0, 2000.0, 5000.0)
    assert x.default_eff == 0.0 and x.effs == [(B2, 1.0)]
    # the species on both sides of a three-molecule side is the only collider
    x = m.kin(5)
    assert x.kind == "third" and x.default_eff == 0.0 and x.effs == [(A2B, 1.0)]
    assert sorted(r[5][0]) == [(A, 1), (B2, 1)] and sorted(r[5][1]) == [(B, 1), (AB, 1)]
    assert r[6][:2] == r[7][:2] and r[6][2:] != r[7][2:]


@pytest.mark.parametrize("bad,msg", [
    ("A+B<=>AB  1e13 0 0\n   PLOG / 1.0 1e13 0 0 /", "not supported"),
    ("A+B<=>AB  1e13 0 0\n   REV / 1e12 0 0 /", "not supported"),
    ("A+C<=>AB  1e13 0 0", "unknown species"),
    ("A+A+A<=>A2+A  1e13 0 0", None),
    ("A+B+B2<=>AB+A2  1e13 0 0", "more than two molecules"),
    ("A+B<=>AB  1e13 0 0\n   LOW / 1e16 0 0 /", "not a fall-off"),
    ("A+B(+M)<=>AB(+M)  1e13 0 0", "without LOW"),
    ("A+B<=>AB  1e13 0 0\n   A2/2.0/", "without a third body"),
])
def test_rejected_forms(bad, msg):
    text = "ELEMENTS H O END\nSPECIES A B AB A2 B2 A2B END\n" + _thermo_block() + "REACTIONS\n" + bad + "\nEND\n"
    if msg is None:   # 3 A <=> A2 + A: A is on both sides -> A + A <=> A2 with collider A
        m = parse_chemkin(text)
        assert m.kin(0).kind == "third" and m.kin(0).effs == [(0, 1.0)]
        assert m.reactions[0][:2] == ([(0, 2)], [(3, 1)])
        return
    with pytest.raises(ChemkinError, match=msg):
        parse_chemkin(text)


def test_converted_mechanism_runs_in_the_oracle(tmp_path, oracle_lib):
    """The H2R stand-in through CHEMKIN text and back gives the oracle the
    same right-hand side (to the precision of the thermo records)."""
    m = standard_mechanism("H2R")
    b = parse_chemkin(to_chemkin(m))
    pa, pb = str(tmp_path / "a.mech"), str(tmp_path / "b.mech")
    m.write(pa)
    b.write(pb)
    oa, ob = oracle_lib.OracleMech(pa), oracle_lib.OracleMech(pb)
    rng = np.random.default_rng(5)
    for _ in range(10):
        y = np.append(rng.dirichlet(np.ones(m.K)), rng.uniform(900, 2400))
        fa, fb = oa.rhs(101325.0, y), ob.rhs(101325.0, y)
        assert np.allclose(fa, fb, rtol=1e-5, atol=1e-12 * np.abs(fa).max())
