"""The C ABI library loads and exports every entry point include/chem.h
declares; argument checks that need no GPU return the documented codes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "chem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chem_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("chem_load_mechanism", "chem_integrate", "chem_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2312_13513_amd import chem
    lib = chem.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(chem.EXPORTED)


def test_default_opts():
    from paper_2312_13513_amd import chem
    o = chem.chem_default_opts()
    assert o.rtol == 1e-8 and o.atol == 1e-12 and o.max_steps == 20000
    assert o.precision == 0 and o.schedule == -1 and o.qmax == 0


def test_bad_mechanism_files_are_rejected(tmp_path, mech_dir):
    from paper_2312_13513_amd import chem
    bad = tmp_path / "bad.mech"
    bad.write_text("CHEMMECH 2\n")
    with pytest.raises(chem.ChemError) as e:
        chem.chem_load_mechanism(str(bad))
    assert e.value.code == -4
    text = (mech_dir / "M9.mech").read_text().splitlines()
    # break the element balance of the first reaction: swap a product index
    for i, line in enumerate(text):
        if line.startswith("R0 "):
            tok = line.split()
            nr = int(tok[1])
            pos = 2 + 2 * nr + 1
            tok[pos] = str((int(tok[pos]) + 1) % 9)
            text[i] = " ".join(tok)
            break
    unbal = tmp_path / "unbal.mech"
    unbal.write_text("\n".join(text) + "\n")
    with pytest.raises(chem.ChemError) as e:
        chem.chem_load_mechanism(str(unbal))
    assert e.value.code == -4 and "balanced" in str(e.value)
    with pytest.raises(chem.ChemError):
        chem.chem_load_mechanism(str(tmp_path / "missing.mech"))


def test_null_handle_is_rejected():
    from paper_2312_13513_amd import chem
    rc = chem.lib().chem_integrate(None, None, None, None, 0, 10, 1e-6, None, None, None, None)
    assert rc == -1
    assert b"NULL" in chem.lib().chem_last_error()


def test_stats_argument_checks():
    """chem_get_stats rejects a NULL result and a negative size before any
    device work."""
    from paper_2312_13513_amd import chem
    out = chem.chem_stats()
    lib = chem.lib()
    assert lib.chem_get_stats(None, None, 4, None, None, None) == -1
    assert lib.chem_get_stats(None, None, -1, None, C.byref(out), None) == -1
