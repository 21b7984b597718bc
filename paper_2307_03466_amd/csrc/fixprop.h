// Host fix-and-propagate rounding (Section 2.3) of the pump loop.
#pragma once

#include <stdint.h>

#include <vector>

namespace scy {

// One LP with local indices: CSR rows, column incidence (cptr / crow, built
// by build_incidence), right-hand side, senses and bounds.
struct FPProblem {
    int32_t m = 0, n = 0;
    const int32_t *ptr = nullptr;   // [m + 1]
    const int32_t *col = nullptr;   // [nnz]
    const double *val = nullptr;    // [nnz]
    const double *b = nullptr;      // [m]
    const char *sense = nullptr;    // [m]
    const double *l = nullptr, *u = nullptr;  // [n]
    const int32_t *cptr = nullptr;  // [n + 1]
    const int32_t *crow = nullptr;  // rows of each column, increasing
    const double *cval = nullptr;   // a_ij of each (column, row) incidence
};

// Everything one visit of a row reads, in one 48-byte record.
struct FPRow {
    double lo = 0.0, hi = 0.0;     // finite parts of min / max activity (exact mode)
    double b = 0.0;
    double reach = 0.0;            // exact mode: an upper bound of max_j |a_ij| (U_j - L_j)
    int32_t lo_inf = 0, hi_inf = 0;  // infinite contributions to min / max activity
    char sense = 'E';
    uint8_t ignored = 0, queued = 0;
};

struct FPDomain {
    double L, U;
};

// The part of the rounding's state that does not depend on the reference
// point: starting domains (integer bounds rounded inward), row records with
// their starting activities, and whether all data are integers (exact mode).
struct FPPrep {
    std::vector<FPRow> rows;
    std::vector<FPDomain> dom;
    int32_t maxlen = 1;
    bool exact = false;
    bool ready = false;
};

void build_incidence(FPProblem &P, std::vector<int32_t> &cptr, std::vector<int32_t> &crow,
                     std::vector<double> &cval);

// Every row holds at x within tol * (1 + |b_i|).
bool rows_satisfied(const FPProblem &P, const double *x, double tol);

// Fills prep for P and is_int (once per problem; reused by every rounding).
void fp_prepare(const FPProblem &P, const uint8_t *is_int, FPPrep &prep);

// Rounds xref to xhat; *feasible = every row satisfied by xhat (1e-6
// relative), *ignored = rows ignored by the propagation.  prep must come
// from fp_prepare on the same P and is_int.
void fix_and_propagate(const FPProblem &P, const uint8_t *is_int, const FPPrep &prep, const double *xref,
                       double *xhat, int32_t *feasible, int32_t *ignored);

}  // namespace scy
