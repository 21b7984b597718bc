// Test driver for the library's host fix-and-propagate (no GPU): reads one
// LP, its integer flags and a reference point from a binary file, rounds it
// with the library's sequential procedure and writes the rounding, the
// feasibility flag and the number of ignored rows.  Unlike the C entry
// point it does not reject non-finite reference values, so the tests can
// reach the rounding's handling of a failed solve's iterate.  Built with
// AddressSanitizer / UBSan by the tests.
//
// Input:  int32 m, n; int64 nnz; int64 row_ptr[m+1]; int32 col_idx[nnz];
//         double val[nnz], b[m]; uint8 sense[m]; double l[n], u[n];
//         uint8 is_int[n]; double x_ref[n].
// Output: double x_hat[n]; int32 feasible, ignored.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2307_03466_amd/csrc/fixprop.h"

template <class T>
static std::vector<T> rd(FILE *f, size_t n)
{
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return v;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 1;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t mn[2];
    int64_t nnz;
    if (fread(mn, 4, 2, f) != 2 || fread(&nnz, 8, 1, f) != 1) return 2;
    const int32_t m = mn[0], n = mn[1];
    auto rp = rd<int64_t>(f, (size_t)m + 1);
    auto col = rd<int32_t>(f, (size_t)nnz);
    auto val = rd<double>(f, (size_t)nnz);
    auto b = rd<double>(f, (size_t)m);
    auto sense = rd<char>(f, (size_t)m);
    auto l = rd<double>(f, (size_t)n);
    auto u = rd<double>(f, (size_t)n);
    auto is_int = rd<uint8_t>(f, (size_t)n);
    auto xref = rd<double>(f, (size_t)n);
    fclose(f);

    std::vector<int32_t> ptr(m + 1), cptr, crow;
    std::vector<double> cval;
    for (int32_t i = 0; i <= m; ++i) ptr[i] = (int32_t)rp[i];
    scy::FPProblem P;
    P.m = m;
    P.n = n;
    P.ptr = ptr.data();
    P.col = col.data();
    P.val = val.data();
    P.b = b.data();
    P.sense = sense.data();
    P.l = l.data();
    P.u = u.data();
    scy::build_incidence(P, cptr, crow, cval);
    scy::FPPrep prep;
    scy::fp_prepare(P, is_int.data(), prep);
    std::vector<double> xhat(n);
    int32_t feas = 0, ign = 0;
    scy::fix_and_propagate(P, is_int.data(), prep, xref.data(), xhat.data(), &feas, &ign);

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 6;
    fwrite(xhat.data(), 8, (size_t)n, o);
    fwrite(&feas, 4, 1, o);
    fwrite(&ign, 4, 1, o);
    fclose(o);
    return 0;
}
