// Kernel argument blocks and host launchers of the PDHG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "scylla_internal.h"

namespace scy {

enum { DIR_ROW = 0, DIR_COL = 1 };

// One orientation of the matrix in device memory.
struct MatView {
    const int32_t *ptr;   // [rows + 1]
    const uint32_t *ent;  // [nnz] index or packed word
    const void *val;      // [nnz] values (format dependent) or null
    int32_t shift;        // packed: value = (int32)word >> shift
    uint32_t mask;        // packed: index = word & mask
};

// Arguments of one pass (row pass = dual step over the CSR, column pass =
// primal step over the CSC) and of its FP64 check variant.
template <class V>
struct PassArgs {
    MatView M;
    const int4 *tiles;
    int32_t ntiles;
    const int4 *longs;    // long-row descriptors {row, slot0, nseg, inst}
    int32_t nlong;
    const V *gvec;        // gathered vector: x_bar (row pass), y (column
                          // pass); x (row check)
    V *own;               // y (row) / x (column), updated in place
    V *bar;               // x_bar output (column pass)
    V *own_ref;           // restart reference y_r / x_r
    const V *rhs;         // b (row) / c_hat (column)
    const V *diag2;       // D_r^2 / D_c^2
    const V *lo, *hi;     // l, u (column)
    const V *ibnd;        // [2 * count] (l, u) shared by every column of an
                          // instance, NaN where they differ (column pass)
    const uint8_t *sense; // row senses
    InstState *st;
    V *seg;               // long-row segment partials
    double *seg64;        // long-row segment partials (check)
    // check variant
    const double *rhs64;  // b / c_hat in FP64
    const double *lo64, *hi64;
    const double *d64;    // d_r / d_c
    double *part;         // 4 doubles per tile (blocked: per combine tile)
    double *lpart;        // 4 doubles per long row
    // gather-blocked orientation
    const int32_t *bptr;  // [B * (rows + 1)] block row pointers
    int32_t rows;         // rows of the orientation
    int32_t B;            // number of gather blocks
    V *P;                 // [B * rows] block partial sums
    double *P64;          // [B * rows] block partial sums (check)
    const int4 *ctiles;   // combine tiles {r0, r1, inst, -1}
    int32_t nctiles;
    // LDS-staged pass
    const int32_t *gofs;  // [count + 1] gathered-vector offsets per instance
    const int4 *sub;      // sub-tiles {r0, r1, inst, -1} of the staged tiles
    // LDS-sliced tiles of the staged pass (tile field w = -2): slice s of
    // instance q gathers [g0 + glen*s/S_q, g0 + glen*(s+1)/S_q) from LDS
    MatView X;            // slice-regrouped entries; X.ptr = [xS * (rows + 1)]
    const int4 *xsub;     // sub-tiles of the sliced tiles
    int32_t xS;           // slices of the longest sliced instance
    const int32_t *xSq;   // [count] slices S_q per instance
    V *xP;                // [xS * rows] slice partial sums (s < S_q written)
    const int32_t *bq;    // combine: partial arrays per instance (null: all B)
    // direct staged pass: tiles {r0, r1, inst, lanes per row} of instances
    // whose whole gathered vector sits in LDS (no product buffer)
    const int4 *dtiles;
    int32_t ndtiles;
    // adaptive step sizes: per epilogue workgroup (ipart) or long row
    // (iplong) two FP64 partials -- column pass {|D_c^-1 dx|^2, 0}, row pass
    // {|D_r^-1 dy|^2, dy^T A dx}.  The column pass then writes the move
    // dx = x+ - x (not x_bar) to `bar`, so the row pass's sum is A dx itself
    // (no difference of two large products), and the row pass forms
    // A x_bar = A x + 2 A dx from the running FP64 product `ax`
    // (A x <- A x + A dx; every row check resets it to A x in FP64)
    int32_t adapt;
    double *ipart, *iplong;
    double *ax;
    // diagonal Hessian of a QP objective (column pass / column check), or
    // null: x+ = proj((x + t D_c^2 (A^T y - c)) / (1 + t D_c^2 q))
    const V *q;
    const double *q64;
    // check: the point of the previous check (y / x) and its product (A x /
    // A^T y, FP64); the check reads them for the infeasibility terms and
    // replaces them by the current ones
    V *own_prev;
    double *prod_prev;
    // restart to the average: the running mean of the iterates since the
    // last restart (x_avg in the column pass, y_avg in the row pass), or
    // null; the epilogue folds every new iterate into it
    V *avg;
};

// Step-size update after iteration jw of the window, one workgroup per
// instance (adaptive steps).
struct StepArgs {
    InstState *st;
    const InstInfo *info;
    const double *rip, *cip;  // iteration partials of the row / column pass
    int32_t jw;
};
void launch_step(const StepArgs &a, int count, hipStream_t s);
// Restart to the average: instances whose decision took the average copy it
// over their iterate (and with adaptive steps its A x over the running one).
template <class V>
void launch_take_avg(InstState *st, const InstInfo *info, V *x, V *y, const V *xa, const V *ya, double *ax,
                     const double *axa, int count, hipStream_t s);

// LDS-staged pass: 1024 threads; variant v: nonzeros per thread per
// sub-tile 4 (v = 0, 1) or 8 (v = 2, 3); odd v prefetch the next
// sub-tile's row bounds and epilogue operands as well.
constexpr int SPASS_NT = 1024;
inline int spass_chunk(int variant) { return SPASS_NT * ((variant & 2) ? 8 : 4); }
// Sub-tile descriptors (rows and nonzero ranges) a staged workgroup keeps in
// static LDS, and the static LDS that takes (the dynamic part must leave it).
constexpr int SPASS_DMAX = 64;
constexpr int SPASS_STATIC_LDS = 4 * SPASS_DMAX * 4;
// LDS beyond the vector that its 16-byte-word copy may use (alignment)
constexpr int LDS_COPY_SLACK = 16;

// Fused check window for instances that fit in LDS (k_tiny).
template <class V>
struct TinyArgs {
    MatView R, C;  // CSR and CSC (normal layout)
    V *x, *xbar, *xr, *y, *yr;
    const V *c, *l, *u, *dc2, *b, *dr2;
    const uint8_t *sense;
    const double *c64, *l64, *u64, *b64, *dr64, *dc64;
    const V *q;           // diagonal Hessian or null
    const double *q64;
    V *xp, *yp;           // point of the previous check
    double *axp, *atyp;   // its products A x, A^T y
    InstState *st;
    const InstInfo *info;
    int32_t adapt;  // adaptive step sizes
};

// LDS bytes k_tiny needs for an instance (must match its carving).
inline size_t tiny_lds_bytes(int m, int n, int rnnz, int cnnz, int vb)
{
    auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return al(4 * (size_t)(m + 1)) + al(4 * (size_t)(n + 1)) + al(4 * (size_t)rnnz) + al(4 * (size_t)cnnz) +
           al((size_t)vb * rnnz) + al((size_t)vb * cnnz) + 8 * al((size_t)vb * n) + 4 * al((size_t)vb * m) +
           al(8 * (size_t)m) + al((size_t)m);
}

template <class V>
void launch_tiny(const TinyArgs<V> &a, int fmt, int count, int R, size_t shmem, hipStream_t s, bool prepare);

struct DecideArgs {
    InstState *st;
    const InstInfo *info;
    const double *rpart, *lrpart, *cpart, *lcpart;
    int32_t R;
    // check partials of the running averages (restart to the average), or null
    const double *rpart2, *lrpart2, *cpart2, *lcpart2;
};

// One pass (or its FP64 check variant): the tile kernel, the long-row
// combine, and for a gather-blocked orientation the row combine.
template <class V>
void launch_pass(const PassArgs<V> &p, int fmt, int dir, int ept, int jw, bool check, bool blocked,
                 hipStream_t s);
// LDS-staged pass over staged tiles {sub0, sub1, inst, -1} (ranges of
// sub-tiles); shmem = product buffer + largest staged vector, in bytes.  prepare = true only raises the
// kernel's dynamic-LDS limit (call once before launching or capturing).
template <class V>
void launch_staged(const PassArgs<V> &p, int fmt, int dir, int variant, int jw, size_t shmem, hipStream_t s,
                   bool prepare);
// Direct staged pass over p.dtiles (k_dpass, 1024 threads, `shmem` bytes of
// dynamic LDS = the largest gathered vector); prepare = true only raises the
// kernel's dynamic-LDS limit.
constexpr int DPASS_NT = 1024;
template <class V>
void launch_direct(const PassArgs<V> &p, int fmt, int dir, int k, int jw, size_t shmem, hipStream_t s,
                   bool prepare);
// Row combine of the LDS-sliced tiles: p.ctiles / p.nctiles / p.B / p.P set
// to the sliced plan's combine tiles, slice count and partials.
template <class V>
void launch_combine(const PassArgs<V> &p, int dir, int jw, hipStream_t s);
void launch_decide(const DecideArgs &d, int count, hipStream_t s);
void launch_force_stop(InstState *st, int count, hipStream_t s);
// flag |= 1 if x[0, n) holds a NaN, |= 2 if y[0, m) holds a non-finite value
// (either pointer may be null; *flag must start at 0).
void launch_start_check(const double *x, int n, const double *y, int m, int *flag, hipStream_t s);
void launch_scale_reduce(const MatView &M, int fmt, int rows, const double *drow, const double *dcol,
                         double *out, int mode, hipStream_t s);
void launch_scale_apply(double *d, const double *r, int len, hipStream_t s);
void launch_inst_norms(const InstInfo *info, int count, const double *b, const double *c,
                       const double *dr, const double *dc, InstState *st, hipStream_t s);
template <class V>
void launch_finish_diag(const double *d, V *d2, int len, hipStream_t s);
template <class V>
void launch_cast(const double *src, V *dst, int len, hipStream_t s);
template <class V>
void launch_project(V *x, const V *l, const V *u, int clo, int chi, V *y, const uint8_t *sense, int rlo,
                    int rhi, int zero, hipStream_t s);
template <class V>
void launch_blend(const double *c_orig, const uint8_t *xbits, const uint8_t *ibits, double a, double kappa,
                  double *c64, V *cv, int lo, int hi, hipStream_t s);
// MIP-feasibility of x per instance (rows within tol (1 + |b_i|), bounds
// and integrality within tol): rbad [m], cbad [n] scratch flags,
// feasible [count] = 1 / 0.
template <class V>
void launch_mip_check(const MatView &M, int fmt, int m, int n, int count, const InstInfo *info, const V *x,
                      const double *b, const uint8_t *sense, const double *l, const double *u,
                      const uint8_t *is_int, double tol, uint8_t *rbad, uint8_t *cbad, uint8_t *feasible,
                      hipStream_t s);

}  // namespace scy
