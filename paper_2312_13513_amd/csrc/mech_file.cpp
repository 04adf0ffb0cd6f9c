// Reader of the text mechanism format; see mech_file.h.

#include "mech_file.h"

#include <cmath>
#include <fstream>
#include <sstream>

#include "chem.h"

namespace chem_file {

namespace {

// Whitespace-token reader with error reporting.
class Tokens {
  public:
    explicit Tokens(std::istream &in) : in_(in) {}
    bool word(std::string &w) { return static_cast<bool>(in_ >> w); }
    bool expect(const char *w)
    {
        std::string s;
        return word(s) && s == w;
    }
    template <typename T>
    bool num(T &v)
    {
        std::string s;
        if (!word(s)) return false;
        std::istringstream is(s);
        is >> v;
        return !is.fail() && is.eof();
    }

  private:
    std::istream &in_;
};

// Version 2 tail of a reaction line: reversibility flag, kind, the
// low-pressure triple and Troe parameters of the fall-off kinds, then the
// default and listed third-body efficiencies of the pressure-dependent kinds.
int parse_kinetics(Tokens &t, int K, int i, HostRxn &r, std::string &err)
{
    const std::string at = " of reaction " + std::to_string(i);
    auto fail = [&](const std::string &msg) {
        err = msg + at;
        return CHEM_EMECH;
    };
    int rev = -1;
    std::string kind;
    if (!t.num(rev) || (rev != 0 && rev != 1) || !t.word(kind)) return fail("bad kinetics tail");
    r.reversible = rev == 1;
    static const char *const names[] = {"elem", "third", "lind", "troe3", "troe4"};
    r.kind = -1;
    for (int k = 0; k < 5; k++)
        if (kind == names[k]) r.kind = k;
    if (r.kind < 0) return fail("unknown reaction kind '" + kind + "'");
    if (r.kind == kElem) return CHEM_OK;
    if (r.kind >= kLind &&
        (!t.num(r.A0) || !t.num(r.b0) || !t.num(r.Ea0) || !(r.A0 > 0) || !std::isfinite(r.A0) ||
         !std::isfinite(r.b0) || !std::isfinite(r.Ea0)))
        return fail("bad low-pressure Arrhenius data");
    const int ntroe = r.kind == kTroe3 ? 3 : (r.kind == kTroe4 ? 4 : 0);
    for (int j = 0; j < ntroe; j++)
        if (!t.num(r.troe[j]) || !std::isfinite(r.troe[j])) return fail("bad Troe parameters");
    if (ntroe && !(r.troe[1] > 0 && r.troe[2] > 0)) return fail("Troe temperatures T3 and T1 must be > 0");
    int n = -1;
    if (!t.num(r.default_eff) || !(r.default_eff >= 0) || !std::isfinite(r.default_eff) || !t.num(n) || n < 0 ||
        n > K)
        return fail("bad third-body efficiencies");
    std::vector<char> seen((size_t)K, 0);
    for (int j = 0; j < n; j++) {
        int k = -1;
        double e = -1;
        if (!t.num(k) || !t.num(e) || k < 0 || k >= K || !(e >= 0) || !std::isfinite(e) || seen[(size_t)k])
            return fail("bad third-body efficiency");
        seen[(size_t)k] = 1;
        r.effs.push_back({k, e});
    }
    return CHEM_OK;
}

}  // namespace

int parse_mech(std::istream &in, HostMech &m, std::string &err)
{
    auto fail = [&err](int code, const std::string &msg) {
        err = msg;
        return code;
    };
    Tokens t(in);
    int ver = 0, seed = 0, attempt = 0;
    std::string gen, u;
    if (!t.expect("CHEMMECH") || !t.num(ver) || (ver != 1 && ver != 2))
        return fail(CHEM_EMECH, "not a CHEMMECH 1 or 2 file");
    if (!t.expect("generator") || !t.word(gen) || !t.expect("seed") || !t.num(seed) ||
        !t.expect("attempt") || !t.num(attempt) || !t.expect("units"))
        return fail(CHEM_EMECH, "bad header");
    for (int i = 0; i < 6; i++)
        if (!t.word(u)) return fail(CHEM_EMECH, "bad units line");
    if (!t.expect("elements") || !t.num(m.E) || m.E < 1 || m.E > 16)
        return fail(CHEM_EMECH, "bad element count");
    m.aw.resize(m.E);
    for (int e = 0; e < m.E; e++) {
        std::string name;
        if (!t.word(name) || !t.num(m.aw[e]) || !(m.aw[e] > 0))
            return fail(CHEM_EMECH, "bad element record");
    }
    if (!t.expect("species") || !t.num(m.K) || m.K < 1 || m.K > 4096)
        return fail(CHEM_EMECH, "bad species count");
    m.counts.assign(m.K, std::vector<int>(m.E));
    m.nasa.assign(m.K, std::vector<double>(17));
    for (int k = 0; k < m.K; k++) {
        std::string name;
        if (!t.word(name)) return fail(CHEM_EMECH, "truncated species list");
        int atoms = 0;
        for (int e = 0; e < m.E; e++) {
            if (!t.num(m.counts[k][e]) || m.counts[k][e] < 0)
                return fail(CHEM_EMECH, "bad element counts of species " + name);
            atoms += m.counts[k][e];
        }
        if (atoms == 0) return fail(CHEM_EMECH, "species " + name + " has no atoms");
        for (int j = 0; j < 17; j++)
            if (!t.num(m.nasa[k][j]) || !std::isfinite(m.nasa[k][j]))
                return fail(CHEM_EMECH, "bad NASA coefficients of species " + name);
        if (!(m.nasa[k][0] < m.nasa[k][1] && m.nasa[k][1] < m.nasa[k][2]))
            return fail(CHEM_EMECH, "bad NASA temperature ranges of species " + name);
    }
    if (!t.expect("reactions") || !t.num(m.R) || m.R < 0 || m.R > 1000000)
        return fail(CHEM_EMECH, "bad reaction count");
    m.rxn.resize(m.R);
    for (int i = 0; i < m.R; i++) {
        HostRxn &r = m.rxn[i];
        std::string name;
        int n = 0;
        if (!t.word(name) || !t.num(n) || n < 1 || n > 2)
            return fail(CHEM_EMECH, "bad reactant list of reaction " + std::to_string(i));
        for (int s = 0; s < n; s++) {
            int k = -1, nu = 0;
            if (!t.num(k) || !t.num(nu) || k < 0 || k >= m.K || nu < 1)
                return fail(CHEM_EMECH, "bad reactant of reaction " + std::to_string(i));
            r.reac.push_back({k, nu});
        }
        if (!t.num(n) || n < 1 || n > 2)
            return fail(CHEM_EMECH, "bad product list of reaction " + std::to_string(i));
        for (int s = 0; s < n; s++) {
            int k = -1, nu = 0;
            if (!t.num(k) || !t.num(nu) || k < 0 || k >= m.K || nu < 1)
                return fail(CHEM_EMECH, "bad product of reaction " + std::to_string(i));
            r.prod.push_back({k, nu});
        }
        if (!t.num(r.A) || !t.num(r.b) || !t.num(r.Ea) || !(r.A > 0) || !std::isfinite(r.b) ||
            !std::isfinite(r.Ea))
            return fail(CHEM_EMECH, "bad Arrhenius data of reaction " + std::to_string(i));
        int mr = 0, mp = 0;
        for (auto &s : r.reac) mr += s.second;
        for (auto &s : r.prod) mp += s.second;
        if (mr > 2 || mp > 2)
            return fail(CHEM_EMECH, "reaction " + std::to_string(i) + " has more than two molecules on a side");
        if (ver == 2) {
            const int rc = parse_kinetics(t, m.K, i, r, err);
            if (rc != CHEM_OK) return rc;
        }
        for (int e = 0; e < m.E; e++) {
            int bal = 0;
            for (auto &s : r.reac) bal -= s.second * m.counts[s.first][e];
            for (auto &s : r.prod) bal += s.second * m.counts[s.first][e];
            if (bal != 0)
                return fail(CHEM_EMECH, "reaction " + std::to_string(i) + " is not element balanced");
        }
    }
    if (!t.expect("end")) return fail(CHEM_EMECH, "missing end marker");
    return CHEM_OK;
}

int parse_mech_file(const char *path, HostMech &m, std::string &err)
{
    std::ifstream f(path);
    if (!f) {
        err = std::string("cannot open mechanism file ") + path;
        return CHEM_EMECH;
    }
    return parse_mech(f, m, err);
}

}  // namespace chem_file
