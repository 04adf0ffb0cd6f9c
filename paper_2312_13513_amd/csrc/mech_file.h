// Reader of the text mechanism format (.mech): species with element counts
// and NASA-7 polynomials, reactions with mass-action Arrhenius rates and (in
// format version 2) third-body, Lindemann or Troe fall-off pressure
// dependence and irreversible reactions.  Plain
// C++17 with no HIP dependency, so it can also be built for the host alone
// (the sanitizer build of the tests does so).
#pragma once

#include <istream>
#include <string>
#include <utility>
#include <vector>

namespace chem_file {

// Pressure dependence of a reaction (format version 2; version 1 files hold
// elementary reversible reactions only).
enum RxnKind { kElem = 0, kThird = 1, kLind = 2, kTroe3 = 3, kTroe4 = 4 };

struct HostRxn {
    std::vector<std::pair<int, int>> reac, prod;   // (species, coefficient)
    double A = 0, b = 0, Ea = 0;                   // A in cm-mol-s, Ea in J/mol
    int kind = kElem;
    bool reversible = true;
    double default_eff = 1.0;                      // third-body efficiency of unlisted species
    std::vector<std::pair<int, double>> effs;      // (species, efficiency), species distinct
    double A0 = 0, b0 = 0, Ea0 = 0;                // low-pressure limit (fall-off kinds)
    double troe[4] = {0, 0, 0, 0};                 // a, T3, T1, T2 (T2: kTroe4 only)
};

struct HostMech {
    int K = 0, R = 0, E = 0;
    std::vector<double> aw;                 // atomic weights, g/mol
    std::vector<std::vector<int>> counts;   // K x E
    std::vector<std::vector<double>> nasa;  // K x 17: Tlow Tmid Thigh, 7 low-range, 7 high-range
    std::vector<HostRxn> rxn;
};

// Parses and validates a whole mechanism.  Returns CHEM_OK, or CHEM_EMECH with
// a message in err; m is then partly filled and must not be used.
int parse_mech(std::istream &in, HostMech &m, std::string &err);
int parse_mech_file(const char *path, HostMech &m, std::string &err);

}  // namespace chem_file
