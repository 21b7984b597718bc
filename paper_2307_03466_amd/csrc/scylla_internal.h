// Internal declarations shared by the host preparation, the kernels and the
// runtime of the PDHG library.  Nothing here is part of the public C ABI.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/scylla_pdhg.h"

namespace scy {

// Matrix storage formats (per handle and orientation).
enum Fmt : int32_t {
    FMT_PACKED = 0,  // 32-bit word: index in the low `shift` bits, signed
                     // integer value in the high bits (0/1 and small-integer
                     // matrices: 4 bytes per nonzero, exact)
    FMT_BF16 = 1,    // int32 index + bfloat16 value (every value BF16-exact)
    FMT_F32 = 2,     // int32 index + float value
    FMT_F64 = 3,     // int32 index + double value (FP64 path)
    FMT_CACHED = 8   // flag on a format given to the pass kernels: matrix
                     // entries are read with plain (cacheable) loads
                     // instead of non-temporal ones
};

enum Status : int32_t { ST_RUN = 0, ST_OPT = 1, ST_ITER = 2, ST_TIME = 3, ST_NUM = 4, ST_PINF = 5, ST_DINF = 6,
                       ST_STALL = 7 };

// Doubles per check partial slot: row pass {|r_p|^2, b^T y, |dy~|^2, -,
// b^T v, |v - proj_Y v|^2, |row violation of A d|^2, -}; column pass
// {|r_d|^2, c^T x (+ x^T Q x / 2), bound terms (- x^T Q x / 2), |dx~|^2,
// |A^T v + lam|^2, ray bound terms, c^T d, |bound violation of d|^2 (+ |Q d|^2)}
// with d, v the moves since the previous check (infeasibility certificates).
constexpr int CHK = 8;

// Per-instance solver state, resident in device memory and updated only by
// the decision kernel (one writer per instance).
struct InstState {
    int32_t status;       // Status
    int32_t nrun;         // iterations to run in the current window
    int32_t restarts;     // restarts taken in this call
    int32_t restart_now;  // 1: copy (x, y) to the restart reference in the
                          //    first iteration of the window
    int32_t restart_on;   // restart scheme enabled
    int32_t force_stop;   // host-requested stop (time limit)
    int32_t avg_on;       // restart to the average: the running mean of the
                          //    iterates since the last restart is a candidate
    int32_t take_avg;     // 1: replace the iterate by that mean before the
                          //    next iteration (set by the decision)
    int64_t k;            // iterations done at the last check
    int64_t k_limit;      // iteration limit of this call
    int64_t kr;           // iteration of the last restart
    int64_t pad2;
    double t, s;          // primal / dual step (eta / omega, eta * omega)
    double omega, eta;
    double tol;
    double Er, Ep;        // KKT error at the last restart / previous check
    double rel, rho_p, rho_d, rho_g, pobj, dobj;
    double bnorm, cnorm;  // ||b||_2, ||c_hat||_2 of the instance
    double omega0;        // primal weight from the data (cold start)
    double infeas_tol;    // > 0: infeasibility certificates at the checks
    double stall_tol;     // > 0: stop when the objective bounds stall
    double pprev, dprev;  // primal / dual objective at the previous check
    int32_t stall_checks; // checks in a row without a move that stop the solve
    int32_t nstall;       // current run of such checks
};

// Static per-instance ranges in the concatenated arrays.
struct InstInfo {
    int32_t row0, row1, col0, col1;  // row / column ranges
    int32_t rt0, rt1, ct0, ct1;      // CSR / CSC tile ranges
    int32_t lr0, lr1, lc0, lc1;      // long-row / long-column ranges
    int32_t ir[2][3][2];             // iteration-partial slot ranges of the
                                     // row / column pass, up to three each
};

// Tile of an orientation: {a, b, inst, slot}.  slot < 0: rows [a, b);
// slot >= 0: nonzeros [a, b) of one long row, partial sum goes to slot.
// Long row descriptor: {row, first slot, number of segments, inst}.

// ----------------------------------------------------------- host side
struct HostOrient {
    int32_t rows = 0;
    std::vector<int32_t> ptr;    // [rows + 1]
    std::vector<uint32_t> ent;   // index or packed word
    std::vector<uint16_t> v16;   // BF16 values
    std::vector<float> v32;      // FP32 values
    std::vector<double> v64;     // FP64 values
    int32_t shift = 0;           // packed: value bits start here
    uint32_t mask = 0xffffffffu; // packed: index mask
};

struct TilePlan {
    int32_t chunk = 0;                 // nonzeros per tile (NT * EPT)
    std::vector<int32_t> tiles;        // 4 ints per tile
    std::vector<int32_t> longs;        // 4 ints per long row
    int32_t nslots = 0;                // segment partial slots
    std::vector<int32_t> t_begin, t_end, l_begin, l_end;  // per instance
};

// Gather-blocked copy of an orientation: the gathered index space is cut
// into B contiguous blocks and every row's nonzeros are regrouped block by
// block (rows stay sorted inside a block).  Block b's nonzeros form one
// contiguous CSR with row pointers bptr[b * (rows + 1) + i].
struct BlockedHost {
    int32_t B = 0;
    std::vector<int32_t> bounds;  // [B + 1] gathered-index boundaries
    std::vector<int32_t> bptr;    // [B * (rows + 1)]
    std::vector<uint32_t> ent;
    std::vector<uint16_t> v16;
    std::vector<float> v32;
    std::vector<double> v64;
};

// Tile list of a blocked orientation, laid out so that workgroup w runs on
// XCD w % 8 and every XCD only touches the gathered slice of one block.
// Tiles carry the block in bits 24.. of the instance field.
struct BlockedPlan {
    int32_t chunk = 0;
    std::vector<int32_t> tiles;   // 4 ints per tile, empty tiles {0,0,0,-1}
    std::vector<int32_t> longs;   // {row, slot0, nseg, inst | block << 24}
    int32_t nslots = 0;
    std::vector<int32_t> ctiles;  // combine tiles {r0, r1, inst, -1}
    std::vector<int32_t> ct_begin, ct_end;  // combine tiles per instance
};

// Plan of an LDS-staged orientation.  Instances whose gathered vector has at
// most max_vec elements and no row longer than sub_chunk get sub-tiles
// (whole rows, <= sub_chunk nonzeros) grouped into ceil(nnz / group_nnz)
// staged tiles per instance of about equal nonzero counts; the other
// instances get normal tiles (rest).
struct StagedPlan {
    std::vector<int32_t> tiles;   // {sub0, sub1, inst, -1}
    TilePlan sub;                 // sub-tiles of the staged instances
    std::vector<uint8_t> staged;  // per instance
    TilePlan rest;                // normal tiles of the other instances
    int32_t max_vec = 0;          // largest staged gathered vector (elements)
};

void plan_staged(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, int32_t max_vec, int32_t sub_chunk, int32_t group_nnz,
                 int32_t rest_chunk, StagedPlan &plan);

// LDS-sliced part of a staged orientation.  An instance whose gathered
// vector is longer than max_vec but at most max_slices * max_vec, with no
// row longer than sub_chunk, has its gathered range cut into
// S_q = ceil(glen / max_vec) equal slices [g0 + glen*s/S_q,
// g0 + glen*(s+1)/S_q); each row's nonzeros are regrouped by slice
// (bptr[s * (rows + 1) + i] points into ent, for s below S = the largest
// S_q; rows of other instances and slices s >= S_q are empty).  Sub-tiles of a slice's rows (<= sub_chunk
// nonzeros, <= 4096 rows) are grouped into ceil(nnz / group_nnz) tiles of
// about equal nonzero counts per (instance, slice)
// {sub0, sub1, inst | s << 24, -2}; the slice partial sums of a row
// are added in slice order by the combine tiles {r0, r1, inst, -1}.
struct SlicedPlan {
    int32_t S = 0;                // slices of the longest sliced instance (0: none)
    std::vector<uint8_t> sliced;  // per instance
    std::vector<int32_t> Sq;      // slices per instance (0: not sliced)
    std::vector<int32_t> bptr;    // [S * (rows + 1)]
    std::vector<uint32_t> ent;
    std::vector<uint16_t> v16;
    std::vector<float> v32;
    std::vector<double> v64;
    std::vector<int32_t> tiles;   // {sub0, sub1, inst | s << 24, -2}
    std::vector<int32_t> sub;     // {r0, r1, inst, -1}, rows of one slice
    std::vector<int32_t> ctiles;  // {r0, r1, inst, -1}
    int32_t max_slice = 0;        // longest slice (elements)
};

// Instances with `candidate[q]` set are considered for slicing.
// build_sliced chooses S and the instances and regroups their entries;
// tile_sliced builds the tiles (cheap; redone per tile size); plan_sliced
// does both.
void build_sliced(const HostOrient &o, int32_t fmt, const std::vector<int32_t> &inst_off,
                  const std::vector<int32_t> &gofs, const std::vector<uint8_t> &candidate, int32_t max_vec,
                  int32_t max_slices, int32_t sub_chunk, SlicedPlan &plan);
void tile_sliced(const std::vector<int32_t> &inst_off, int32_t rows, int32_t sub_chunk, int32_t group_nnz,
                 SlicedPlan &plan);
void plan_sliced(const HostOrient &o, int32_t fmt, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, const std::vector<uint8_t> &candidate, int32_t max_vec,
                 int32_t max_slices, int32_t sub_chunk, int32_t group_nnz, SlicedPlan &plan);

// Nonzeros per lane per row and round of the direct staged pass for a plan
// with at least L lanes per row (rows of up to 16 nonzeros take one round).
inline int32_t dpass_k(int32_t L) { return L <= 2 ? 8 : (L <= 4 ? 4 : 2); }

// Direct staged tiles: every instance with rows and a gathered vector of at
// most max_vec elements (direct[q] = 1) has its rows cut into runs of whole
// rows with about group_nnz nonzeros, tiles {r0, r1, q, L}: L lanes per row,
// the smallest power of two >= lanes_min (at most 64) for which the tile's
// longest row takes at most four rounds of per_lane nonzeros per lane.
void plan_direct(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, int32_t max_vec, int32_t group_nnz, int32_t lanes_min,
                 int32_t per_lane, std::vector<uint8_t> &direct, std::vector<int32_t> &tiles);

void build_blocked(const HostOrient &o, int32_t fmt, int32_t gather_size, int32_t B, BlockedHost &out);
void plan_blocked(const BlockedHost &bh, int32_t rows, const std::vector<int32_t> &inst_off, int32_t chunk,
                  int32_t max_rows, BlockedPlan &plan);

// Validation of one LP description (no GPU).  Returns 0 or -EINVAL.
int validate_lp(const scylla_lp *lp, std::string &err);

// Concatenates `count` LPs into one block-diagonal CSR and its CSC copy,
// choosing the storage format (FMT_F64 for the FP64 path; for FP32 the most
// compact exact one).  Row/column offsets per instance are returned.
int build_orientations(const scylla_lp *lps, int32_t count, int32_t precision, HostOrient &csr,
                       HostOrient &csc, int32_t &fmt, std::vector<int32_t> &row_off,
                       std::vector<int32_t> &col_off, std::string &err);

// Splits the rows of an orientation into tiles of at most `chunk` nonzeros
// and at most `max_rows` rows; rows longer than `chunk` become long rows cut
// into `chunk`-sized segments.  Tiles never straddle instances.
void plan_tiles(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                int32_t chunk, int32_t max_rows, TilePlan &plan, const uint8_t *skip = nullptr);

uint16_t f64_to_bf16_exact(double v, bool &exact);

}  // namespace scy
