"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The library's two file readers (mechanism text files, surrogate weight and
checkpoint files) are plain C++ with no HIP dependency, and the oracle is plain
C; both are built here with -fsanitize=address,undefined and run on valid
files and on damaged ones (truncated, tokens replaced by junk or extreme
values, header fields set to extreme values with the checksum made good
again).  Every run must end normally with no sanitizer report; damaged files
must be rejected where the damage makes them invalid, and a surrogate file
that decodes must encode back to the same bytes."""
import os
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_13513_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=86", UBSAN_OPTIONS="print_stacktrace=1:exitcode=87")


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    host, orc = d / "host_files", d / "oracle_main"
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(HERE, "host_files_main.cpp"), os.path.join(CSRC, "mech_file.cpp"),
                    os.path.join(CSRC, "surr_file.cpp"), "-o", str(host)], check=True)
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", os.path.join(HERE, "oracle_main.c"),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", str(orc)], check=True)
    return host, orc


def run(*cmd):
    r = subprocess.run([str(c) for c in cmd], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (cmd[:3], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout.splitlines()


def damaged_mechs(text: str, d):
    """(path, must_reject) for damaged copies of a mechanism file."""
    d.mkdir(exist_ok=True)
    toks = text.split()
    out = []

    def put(name, body, must):
        p = d / f"{name}.mech"
        p.write_text(body)
        out.append((p, must))

    for i, cut in enumerate(sorted({0, 1, 3, 7, 12, len(toks) // 4, len(toks) // 2, len(toks) - 2, len(toks) - 1})):
        put(f"cut{i}", " ".join(toks[:cut]), True)
    junk = ["x", "-1", "0", "1e999", "nan", "-inf", "2147483648", "99999999999999999999", "4097", "-2147483649"]
    step = max(1, len(toks) // 37)
    for i in range(0, len(toks), step):
        for j, w in enumerate(junk[(i // step) % 3::3]):
            t = list(toks)
            t[i] = w
            put(f"rep{i}_{j}", " ".join(t), False)
    for key, vals in (("elements", ["0", "17", "-3"]), ("species", ["0", "4097", "100000000"]),
                      ("reactions", ["-1", "1000001", "2000000000"])):
        at = toks.index(key) + 1
        for j, v in enumerate(vals):
            t = list(toks)
            t[at] = v
            put(f"{key}{j}", " ".join(t), True)
    return out


def test_mechanism_readers_under_sanitizers(bins, mech_dir, tmp_path):
    host, orc = bins
    good = [mech_dir / f"{n}.mech" for n in ("M9", "M35", "H2R", "CH4R")]
    want = ["ok 9 21 3", "ok 35 200 4", "ok 9 12 3", "ok 20 85 4"]
    assert run(host, "mech", *good) == want
    lines = run(orc, *good)
    assert all(ln.startswith(w + " ") for ln, w in zip(lines, want))
    cases = damaged_mechs((mech_dir / "M9.mech").read_text(), tmp_path / "m9")
    cases += damaged_mechs((mech_dir / "H2R.mech").read_text(), tmp_path / "h2r")
    got_lib = run(host, "mech", *[p for p, _ in cases])
    got_orc = run(orc, *[p for p, _ in cases])
    assert len(got_lib) == len(got_orc) == len(cases)
    for (p, must), a, b in zip(cases, got_lib, got_orc):
        if must:
            assert a.startswith("rejected"), (p.name, a)
            assert b == "rejected", (p.name, b)
    assert sum(a.startswith("rejected") for a in got_lib) > len(cases) // 2


def fnv1a(b: bytes) -> int:
    h = 0xCBF29CE484222325
    for c in b:
        h = ((h ^ c) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def resealed(body: bytes) -> bytes:
    return body + struct.pack("<Q", fnv1a(body))


def test_surrogate_file_reader_under_sanitizers(bins, tmp_path):
    host, _ = bins
    files = []
    for opt in (0, 1):
        p = tmp_path / f"good{opt}.surr"
        run(host, "surr-write", p, 9, 24, 16, 8, opt, 100)
        files.append(p)
    assert run(host, "surr", *files) == ["ok 9 11 24 16 8 opt=0 user=0", "ok 9 11 24 16 8 opt=1 user=100"]
    cases = []
    for opt, p in enumerate(files):
        raw = p.read_bytes()
        body = raw[:-8]
        # truncated, with and without a good checksum
        for i, cut in enumerate((0, 7, 8, 12, 40, 64, len(raw) // 2, len(raw) - 9, len(raw) - 1)):
            q = tmp_path / f"t{opt}_{i}.surr"
            q.write_bytes(raw[:cut])
            cases.append((q, True))
            if 8 <= cut <= len(body):
                q = tmp_path / f"ts{opt}_{i}.surr"
                q.write_bytes(resealed(body[:cut]))
                cases.append((q, True))
        # header fields (version, six dims, nset, nn) set to extreme values, resealed
        # (offset, format, values that leave the file valid)
        fields = [(8, "<i", ()), *[(12 + 4 * k, "<i", ()) for k in range(6)], (44, "<i", (0,)), (48, "<q", ())]
        nn = struct.unpack_from("<q", body, 48)[0]
        np_at = 56 + 8 * nn
        fields.append((np_at, "<q", ()))
        if opt:
            npar = struct.unpack_from("<q", body, np_at)[0]
            at_t = np_at + 8 + 4 * npar
            fields += [(at_t, "<q", (2**40, 2**62)), (at_t + 8 + 8 * npar, "<q", ())]
        for j, (at, fmt, valid) in enumerate(fields):
            for k, v in enumerate((0, -1, 3, 2**31 - 1) if fmt == "<i" else (-1, 2**40, 2**62)):
                b = bytearray(body)
                struct.pack_into(fmt, b, at, v)
                q = tmp_path / f"f{opt}_{j}_{k}.surr"
                q.write_bytes(resealed(bytes(b)))
                cases.append((q, v not in valid))
        # a byte flipped without resealing: the checksum must catch it
        for i in range(0, len(body), max(1, len(body) // 13)):
            b = bytearray(raw)
            b[i] ^= 0x5A
            q = tmp_path / f"x{opt}_{i}.surr"
            q.write_bytes(bytes(b))
            cases.append((q, True))
    got = run(host, "surr", *[p for p, _ in cases])
    assert len(got) == len(cases)
    for (p, must), line in zip(cases, got):
        if must:
            assert line.startswith("rejected"), (p.name, line)


def test_checkpoint_user_bytes_through_the_c_abi(bins, tmp_path):
    """chem_surrogate_checkpoint_user is host-only: read the caller's bytes of
    a version 2 file through the library (no GPU needed), and refuse a
    version 1 file."""
    host, _ = bins
    from paper_2312_13513_amd import chem
    p2, p1 = tmp_path / "c2.surr", tmp_path / "c1.surr"
    run(host, "surr-write", p2, 9, 24, 16, 8, 1, 100)
    run(host, "surr-write", p1, 9, 24, 16, 8, 0, 0)
    assert chem.Surrogate.checkpoint_user(str(p2)) == b"u" * 100
    with pytest.raises(chem.ChemError, match="no training state"):
        chem.Surrogate.checkpoint_user(str(p1))
