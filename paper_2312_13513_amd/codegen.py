"""Mechanism compiler: emits gfx950 HIP source specialised to one mechanism.

For a given ``.mech`` file it writes a functor whose right-hand side and
analytic Jacobian are straight-line code: species indices, stoichiometry and
Arrhenius/NASA coefficients become compile-time constants, so the kernels do
no table lookups and keep every per-species quantity in registers.  The
functor plugs into the same BDF driver as the table-driven path; the library
picks the specialised kernel when the loaded file's FNV-1a hash matches.

The arithmetic is the same as the table-driven kernels (NASA-7 with
pre-divided coefficients, ln k_f = ln A + b ln T - Ea/(R T), k_r = k_f / K_c
via exp(ln k_f + dG/RT - dnu ln(p0/(R T))), third-body and fall-off factors
from kinetics.h with the efficiencies and low-pressure records as constants).
"""
from __future__ import annotations

import math
import os
import sys
from typing import Dict, List, Tuple

RU = 8.31446261815324
PSTD = 101325.0


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def _read(path: str):
    tok = open(path).read().split()
    pos = [0]

    def nxt():
        pos[0] += 1
        return tok[pos[0] - 1]

    assert nxt() == "CHEMMECH"
    version = nxt()
    assert version in ("1", "2")
    for _ in range(6):
        nxt()
    assert nxt() == "units"
    for _ in range(6):
        nxt()
    assert nxt() == "elements"
    E = int(nxt())
    aw = []
    for _ in range(E):
        nxt()
        aw.append(float(nxt()))
    assert nxt() == "species"
    K = int(nxt())
    counts, nasa = [], []
    for _ in range(K):
        nxt()
        counts.append([int(nxt()) for _ in range(E)])
        nasa.append([float(nxt()) for _ in range(17)])
    assert nxt() == "reactions"
    R = int(nxt())
    rx, kins = [], []
    for _ in range(R):
        nxt()
        nr = int(nxt())
        reac = [(int(nxt()), int(nxt())) for _ in range(nr)]
        npr = int(nxt())
        prod = [(int(nxt()), int(nxt())) for _ in range(npr)]
        A, b, Ea = float(nxt()), float(nxt()), float(nxt())
        rx.append((reac, prod, A, b, Ea))
        kin = {"rev": True, "kind": "elem"}
        if version == "2":
            kin["rev"] = nxt() == "1"
            kin["kind"] = nxt()
            if kin["kind"] in ("lind", "troe3", "troe4"):
                kin["low"] = (float(nxt()), float(nxt()), float(nxt()))
            if kin["kind"] in ("troe3", "troe4"):
                kin["troe"] = [float(nxt()) for _ in range(3 if kin["kind"] == "troe3" else 4)]
            if kin["kind"] != "elem":
                kin["def"] = float(nxt())
                kin["effs"] = [(int(nxt()), float(nxt())) for _ in range(int(nxt()))]
        kins.append(kin)
    assert nxt() == "end"
    W = [1e-3 * sum(c * w for c, w in zip(cnt, aw)) for cnt in counts]
    return K, R, W, nasa, rx, kins


def _lit(x: float) -> str:
    r = repr(float(x))
    if "e" not in r and "." not in r and "inf" not in r and "nan" not in r:
        r += ".0"
    return r


def _range_coefs(a):
    return [a[0], a[1], a[2], a[3], a[4], a[5], a[6],
            a[1] / 2.0, a[2] / 3.0, a[3] / 4.0, a[4] / 5.0, a[2] / 2.0, a[3] / 3.0, a[4] / 4.0]


def _thermo_lines(K, nasa, want_dcp: bool) -> List[str]:
    L = []
    for k in range(K):
        lo, hi = _range_coefs(nasa[k][3:10]), _range_coefs(nasa[k][10:17])
        if lo == hi:
            c = [_lit(v) for v in lo]
        else:
            L.append(f"    const bool lo{k} = T < {_lit(nasa[k][1])};")
            c = [f"(lo{k} ? {_lit(a)} : {_lit(b)})" for a, b in zip(lo, hi)]
        L.append(f"    const double cp{k} = {c[0]} + T * ({c[1]} + T * ({c[2]} + T * ({c[3]} + T * {c[4]})));")
        L.append(f"    const double h{k} = {c[0]} + T * ({c[7]} + T * ({c[8]} + T * ({c[9]} + T * {c[10]}))) + {c[5]} * invT;")
        L.append(f"    const double g{k} = h{k} - ({c[0]} * lnT + T * ({c[1]} + T * ({c[11]} + T * ({c[12]} + T * {c[13]}))) + {c[6]});")
        if want_dcp:
            L.append(f"    const double dcp{k} = {c[1]} + T * (2.0 * {c[2]} + T * (3.0 * {c[3]} + T * 4.0 * {c[4]}));")
    return L


def _rxn_terms(reac, prod):
    slots_r = [k for k, nu in reac for _ in range(nu)]
    slots_p = [k for k, nu in prod for _ in range(nu)]
    net: Dict[int, int] = {}
    for k in slots_r:
        net[k] = net.get(k, 0) - 1
    for k in slots_p:
        net[k] = net.get(k, 0) + 1
    return slots_r, slots_p, net


def _prod_expr(slots, prefix="C") -> str:
    return " * ".join(f"{prefix}{k}" for k in slots)


def _dprod(slots, s) -> str:
    """d(prod of C over slots)/dC_s as an expression (slots may repeat)."""
    cnt = slots.count(s)
    rest = list(slots)
    rest.remove(s)
    body = " * ".join(f"C{k}" for k in rest) if rest else "1.0"
    return f"{cnt}.0 * {body}" if cnt > 1 else body


def _pdep_lines(kin, K: int, order: int, i: int, deriv: bool) -> List[str]:
    """Third-body concentration M and the pressure-dependence factor pd of a
    pressure-dependent reaction (kinetics.h), efficiencies and the
    low-pressure record as constants."""
    eff = [kin["def"]] * K
    for k, v in kin["effs"]:
        eff[k] = v
    terms = [(f"C{k}" if v == 1.0 else f"{_lit(v)} * C{k}") for k, v in enumerate(eff) if v != 0.0]
    L = [f"const double M = {' + '.join(terms) if terms else '0.0'};"]
    if kin["kind"] == "third":
        L.append("const PdepRate pd{M, 0.0, 1.0};")
        return L
    A0, b0, Ea0 = kin["low"]
    troe = kin.get("troe", [0.0, 1.0, 1.0])
    head = [math.log(A0) + order * math.log(1e-6), b0, Ea0 / RU, troe[0],
            1.0 / troe[1] if kin["kind"] != "lind" else 0.0, 1.0 / troe[2] if kin["kind"] != "lind" else 0.0,
            troe[3] if kin["kind"] == "troe4" else 0.0, 1.0 if kin["kind"] == "troe4" else 0.0]
    L.append(f"const double a{i}[{len(head)}] = {{{', '.join(_lit(v) for v in head)}}};")
    kind = "kRxnLind" if kin["kind"] == "lind" else "kRxnTroe"
    L.append(f"const PdepRate pd = pdep_rate<{'true' if deriv else 'false'}>({kind}, a{i}, M, T, lnT, invT, lnkf, "
             f"{'dlnk' if deriv else '0.0'});")
    return L


def _eff_row(kin, K: int) -> List[float]:
    eff = [kin["def"]] * K
    for k, v in kin["effs"]:
        eff[k] = v
    return eff


def _start_waves(K: int, kins) -> int:
    return 2 if K <= 9 and all(k["kind"] == "elem" for k in kins) else 1


def generate(path: str, tag: str) -> Tuple[str, int, int]:
    """Return (source, K, hash) of the specialised functor and kernels for a file."""
    data = open(path, "rb").read()
    hsh = fnv1a64(data)
    K, R, W, nasa, rx, kins = _read(path)
    N = K + 1
    out = [f"// Generated from {os.path.basename(path)} (FNV-1a {hsh:016x}); do not edit.",
           '#include "bdf_driver.h"', "", "namespace chem {", "namespace {", "",
           f"struct GenMech_{tag} {{", f"    static constexpr int K = {K};",
           # waves per SIMD of the start pass: two where its registers fit
           # 256 (up to 9 species, elementary reactions), else one
           f"    static constexpr int kStartWaves = {_start_waves(K, kins)};", ""]
    ln_c0_const = math.log(PSTD / RU)

    # ---------------- right-hand side
    out.append("    __device__ __forceinline__ void rhs(double p, const double *__restrict__ y, double *__restrict__ f) const")
    out.append("    {")
    out.append(f"        const double T = y[{K}];")
    out.append("        const double invT = 1.0 / T;")
    out.append("        const double lnT = log(T);")
    out += ["    " + s for s in _thermo_lines(K, nasa, False)]
    out.append("        const double sumYW = " + " + ".join(f"y[{k}] * {_lit(1.0 / W[k])}" for k in range(K)) + ";")
    out.append(f"        const double rho = p / ({_lit(RU)} * T * sumYW);")
    for k in range(K):
        out.append(f"        const double C{k} = rho * y[{k}] * {_lit(1.0 / W[k])};")
    out.append("        const double cpm = " + " + ".join(f"y[{k}] * cp{k} * {_lit(1.0 / W[k])}" for k in range(K)) + ";")
    out.append(f"        const double ln_c0 = {_lit(ln_c0_const)} - lnT;")
    for k in range(K):
        out.append(f"        double w{k} = 0.0;")
    for i, (reac, prod, A, b, Ea) in enumerate(rx):
        sr, sp, net = _rxn_terms(reac, prod)
        kin = kins[i]
        pdep = kin["kind"] != "elem"
        order = len(sr)
        lnA = math.log(A) + (order - 1 + (kin["kind"] == "third")) * math.log(1e-6)
        dnu = len(sp) - len(sr)
        dg = " + ".join(f"g{k}" for k in sp) + " - " + " - ".join(f"g{k}" for k in sr)
        out.append(f"        {{   // reaction {i}")
        out.append(f"            const double lnkf = {_lit(lnA)} + {_lit(b)} * lnT - {_lit(Ea / RU)} * invT;")
        lnkr = f"lnkf + ({dg})" + (f" - {float(dnu)!r} * ln_c0" if dnu else "")
        q0 = f"exp(lnkf) * {_prod_expr(sr)}" + (f" - exp({lnkr}) * {_prod_expr(sp)}" if kin["rev"] else "")
        if pdep:
            out += ["            " + ln for ln in _pdep_lines(kin, K, order, i, False)]
            out.append(f"            const double q = ({q0}) * pd.mult;")
        else:
            out.append(f"            const double q = {q0};")
        for k, nu in sorted(net.items()):
            if nu:
                out.append(f"            w{k} += {float(nu)!r} * q;")
        out.append("        }")
    out.append("        const double inv_rho = 1.0 / rho;")
    for k in range(K):
        out.append(f"        f[{k}] = {_lit(W[k])} * w{k} * inv_rho;")
    out.append("        const double heat = " + " + ".join(f"h{k} * w{k}" for k in range(K)) + ";")
    out.append(f"        f[{K}] = -({_lit(RU)} * T) * heat / (rho * ({_lit(RU)} * cpm));")
    out.append("    }")
    out.append("")

    # ---------------- Jacobian
    # Species block accumulated straight into J: J_kl += (W_k/W_l) nu_k dq/dC_l.
    # A C (needed for the density/mean-molar-mass chain rule) follows from the
    # homogeneity of mass action: sum_l C_l dq/dC_l = m_f fwd - m_r rev.
    # Sums over species of per-species reaction sums are taken reaction by
    # reaction instead (sum_k h_k sum_r nu_kr x_r = sum_r x_r dh_r), so only
    # one accumulator per species (sum_r nu_kr (q_r - qh_r)) and four scalars
    # stay live beside J while the reactions are walked.
    out.append("    template <class JA>")
    out.append("    __device__ __forceinline__ void jac(double p, const double *__restrict__ y, JA J) const")
    out.append("    {")
    out.append(f"        const double T = y[{K}];")
    out.append("        const double invT = 1.0 / T;")
    out.append("        const double lnT = log(T);")
    out += ["    " + s for s in _thermo_lines(K, nasa, False)]
    out.append("        const double sumYW = " + " + ".join(f"y[{k}] * {_lit(1.0 / W[k])}" for k in range(K)) + ";")
    out.append("        const double wbar = 1.0 / sumYW;")
    out.append(f"        const double rho = p * wbar / ({_lit(RU)} * T);")
    for k in range(K):
        out.append(f"        const double C{k} = rho * y[{k}] * {_lit(1.0 / W[k])};")
    out.append(f"        const double ln_c0 = {_lit(ln_c0_const)} - lnT;")
    touched = set()
    for i, (reac, prod, *_ ) in enumerate(rx):
        sr, sp, net = _rxn_terms(reac, prod)
        cols = set(sr) | set(sp)
        if kins[i]["kind"] != "elem":
            cols |= {l for l, v in enumerate(_eff_row(kins[i], K)) if v != 0.0}
        for k, nu in net.items():
            if nu:
                for l in cols:
                    touched.add((k, l))
    for k in range(K):
        out.append(f"        double v{k} = 0.0;")
        out.append(f"        J[{k * N + K}] = 0.0;")
    out.append("        double sh = 0.0, shAC = 0.0, shT = 0.0, scp = 0.0;")
    for k in range(K):
        for l in range(K):
            if (k, l) in touched:
                out.append(f"        J[{k * N + l}] = 0.0;")
    for i, (reac, prod, A, b, Ea) in enumerate(rx):
        sr, sp, net = _rxn_terms(reac, prod)
        kin = kins[i]
        pdep, rev_ = kin["kind"] != "elem", kin["rev"]
        order = len(sr)
        lnA = math.log(A) + (order - 1 + (kin["kind"] == "third")) * math.log(1e-6)
        dnu = len(sp) - len(sr)
        dg = " + ".join(f"g{k}" for k in sp) + " - " + " - ".join(f"g{k}" for k in sr)
        dh = " + ".join(f"h{k}" for k in sp) + " - " + " - ".join(f"h{k}" for k in sr)
        dcp = " + ".join(f"cp{k}" for k in sp) + " - " + " - ".join(f"cp{k}" for k in sr)
        out.append(f"        {{   // reaction {i}")
        out.append(f"            const double lnkf = {_lit(lnA)} + {_lit(b)} * lnT - {_lit(Ea / RU)} * invT;")
        lnkr = f"lnkf + ({dg})" + (f" - {float(dnu)!r} * ln_c0" if dnu else "")
        out.append(f"            const double dlnk = ({_lit(b)} + {_lit(Ea / RU)} * invT) * invT;")
        if pdep:
            out += ["            " + ln for ln in _pdep_lines(kin, K, order, i, True)]
            out.append("            const double ekf = exp(lnkf);")
            out.append("            const double kf = ekf * pd.mult;")
            if rev_:
                out.append(f"            const double ekr = exp({lnkr});")
                out.append("            const double kr = ekr * pd.mult;")
        else:
            out.append("            const double kf = exp(lnkf);")
            if rev_:
                out.append(f"            const double kr = exp({lnkr});")
        out.append(f"            const double fwd = kf * {_prod_expr(sr)};")
        out.append(f"            const double rev = {'kr * ' + _prod_expr(sp) if rev_ else '0.0'};")
        out.append("            const double q = fwd - rev;")
        if pdep:
            g0 = f"ekf * {_prod_expr(sr)}" + (f" - ekr * {_prod_expr(sp)}" if rev_ else "")
            out.append(f"            const double G = pd.dM * ({g0});")
        out.append(f"            const double qh = {float(len(sr))!r} * fwd - {float(len(sp))!r} * rev"
                   + (" + G * M;" if pdep else ";"))
        out.append(f"            const double dh = {dh};")
        out.append("            const double dlnkf = dlnk" + (" + pd.dlnT;" if pdep else ";"))
        out.append(f"            const double dlnkr = dlnkf - (dh - {float(dnu)!r}) * invT;")
        out.append("            const double dqT = fwd * dlnkf - rev * dlnkr;")
        out.append("            const double qv = q - qh;")
        out.append("            const double qa = dqT + qv * invT;")
        out.append("            sh += q * dh;")
        out.append("            shAC += qh * dh;")
        out.append("            shT += dh * (dqT - qh * invT);")
        out.append(f"            scp += q * ({dcp});")
        species = sorted(set(sr) | (set(sp) if rev_ else set()))
        for sidx in species:
            terms = []
            if sidx in sr:
                terms.append(f"kf * ({_dprod(sr, sidx)})")
            if sidx in sp and rev_:
                terms.append(f"- kr * ({_dprod(sp, sidx)})")
            out.append(f"            const double dq{sidx} = {' '.join(terms)};")
        effrow = _eff_row(kin, K) if pdep else None
        for k, nu in sorted(net.items()):
            if not nu:
                continue
            out.append(f"            v{k} += {float(nu)!r} * qv;")
            out.append(f"            J[{k * N + K}] += {float(nu)!r} * qa;")
            for sidx in species:
                out.append(f"            J[{k * N + sidx}] += {_lit(nu * W[k] / W[sidx])} * dq{sidx};")
            if pdep:   # through [M]: d q / d C_l += G eff_l
                for l, e in enumerate(effrow):
                    if e != 0.0:
                        out.append(f"            J[{k * N + l}] += {_lit(nu * e * W[k] / W[l])} * G;")
        out.append("        }")
    out.append("        const double gq = wbar / rho;")
    out.append(f"        const double RT = {_lit(RU)} * T;")
    out.append(f"        const double cpm = {_lit(RU)} * (" + " + ".join(f"y[{k}] * cp{k} * {_lit(1.0 / W[k])}" for k in range(K)) + ");")
    dcp_terms = []
    for k in range(K):
        lo, hi = _range_coefs(nasa[k][3:10]), _range_coefs(nasa[k][10:17])
        if lo == hi:
            c = [_lit(v) for v in lo]
        else:
            c = [f"(lo{k} ? {_lit(a)} : {_lit(b2)})" for a, b2 in zip(lo, hi)]
        dcp_terms.append(f"y[{k}] * {_lit(1.0 / W[k])} * ({c[1]} + T * (2.0 * {c[2]} + T * (3.0 * {c[3]} + T * 4.0 * {c[4]})))")
    out.append(f"        const double dcpm = {_lit(RU)} * (" + " + ".join(dcp_terms) + ");")
    out.append("        const double rcp = rho * cpm;")
    out.append("        const double inv_rcp = 1.0 / rcp;")
    out.append("        const double inv_rho = 1.0 / rho;")
    out.append("        const double S = RT * sh;")
    out.append("        const double hAC = shAC;")
    out.append(f"        const double dST = {_lit(RU)} * scp + RT * shT;")
    for k in range(K):
        out.append(f"        J[{k * N + K}] *= {_lit(W[k])} * inv_rho;")
    # temperature row from the accumulated block (before its rank-one term)
    for j in range(K):
        col = [f"{_lit(1.0 / W[k])} * h{k} * J[{k * N + j}]" for k in range(K) if (k, j) in touched]
        colsum = " + ".join(col) if col else "0.0"
        out.append(f"        {{ const double dS = RT * rho * (({colsum}) - gq * {_lit(1.0 / W[j])} * hAC);")
        out.append(f"          const double drcp = rho * {_lit(1.0 / W[j])} * ({_lit(RU)} * cp{j} - cpm * wbar);")
        out.append(f"          J[{K * N + j}] = (-dS + S * drcp * inv_rcp) * inv_rcp; }}")
    # rank-one term of the species block: (W_k/W_j) gq (w_k - AC_k)
    for k in range(K):
        out.append(f"        {{ const double u = {_lit(W[k])} * gq * v{k};")
        for j in range(K):
            if (k, j) in touched:
                out.append(f"          J[{k * N + j}] += u * {_lit(1.0 / W[j])};")
            else:
                out.append(f"          J[{k * N + j}] = u * {_lit(1.0 / W[j])};")
        out.append("        }")
    out.append("        const double drcpT = rho * dcpm - cpm * rho * invT;")
    out.append(f"        J[{K * N + K}] = (-dST + S * drcpT * inv_rcp) * inv_rcp;")
    out.append("    }")
    out.append("};")
    out.append("")
    out.append("}  // namespace")
    out.append("")
    out.append(f"CHEM_DEFINE_GEN_LAUNCHERS(GenMech_{tag}, {tag})")
    out.append("")
    out.append("}  // namespace chem")
    return "\n".join(out) + "\n", K, hsh


def write_generated(mech_paths: Dict[str, str], outdir: str) -> List[str]:
    """Generate one source per mechanism plus the registry; return the paths."""
    os.makedirs(outdir, exist_ok=True)
    files, entries = [], []
    for tag, path in sorted(mech_paths.items()):
        src, K, hsh = generate(path, tag)
        fn = os.path.join(outdir, f"gen_{tag}.hip")
        with open(fn, "w") as fh:
            fh.write(src)
        files.append(fn)
        entries.append((tag, K, hsh))
    reg = ['// Generated registry of mechanism-specialised kernels; do not edit.',
           '#include "bdf_driver.h"', "", "namespace chem {"]
    for tag, K, hsh in entries:
        reg.append(f"CHEM_DECLARE_GEN_LAUNCHERS({tag})")
    reg.append("static const GenEntry kGenEntries[] = {")
    for tag, K, hsh in entries:
        reg.append(f"    {{0x{hsh:016x}ull, {K}, \"{tag}\", &gen_integrate_{tag}, &gen_rhs_{tag}, &gen_jac_{tag}}},")
    if not entries:
        reg.append("    {0ull, 0, \"\", nullptr, nullptr, nullptr},")
    reg.append("};")
    reg.append(f"const GenEntry *gen_registry(int *count) {{ *count = {len(entries)}; return kGenEntries; }}")
    reg.append("}  // namespace chem")
    fn = os.path.join(outdir, "gen_registry.cpp")
    with open(fn, "w") as fh:
        fh.write("\n".join(reg) + "\n")
    files.append(fn)
    return files


if __name__ == "__main__":
    src, K, h = generate(sys.argv[1], "test")
    print(src)
