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

void build_incidence(FPProblem &P, std::vector<int32_t> &cptr, std::vector<int32_t> &crow,
                     std::vector<double> &cval);

// Every row holds at x within tol * (1 + |b_i|).
bool rows_satisfied(const FPProblem &P, const double *x, double tol);

// Rounds xref to xhat; *feasible = every row satisfied by xhat (1e-6
// relative), *ignored = rows ignored by the propagation.
void fix_and_propagate(const FPProblem &P, const uint8_t *is_int, const double *xref, double *xhat,
                       int32_t *feasible, int32_t *ignored);

}  // namespace scy
