// Test driver for the library's host-side preparation (no GPU): reads a
// batch of LPs from a binary file, runs build_orientations and plan_tiles
// (and, when asked, build_blocked / plan_blocked with B blocks and
// plan_staged), and writes the results back as raw arrays for the Python
// checks.  Usage: in out chunk max_rows [B [max_vec sub_chunk group_nnz
// [max_slices]]]; with B < 0: in out chunk max_rows B
// max_vec group_nnz lanes_min (direct staged tiles).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2307_03466_amd/csrc/scylla_internal.h"

template <class T>
static std::vector<T> rd(FILE *f, size_t n)
{
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) { fprintf(stderr, "short read\n"); exit(2); }
    return v;
}
template <class T>
static void wr(FILE *f, const std::vector<T> &v)
{
    long long n = (long long)v.size();
    fwrite(&n, 8, 1, f);
    if (n) fwrite(v.data(), sizeof(T), v.size(), f);
}

int main(int argc, char **argv)
{
    if (argc < 5) return 1;
    FILE *f = fopen(argv[1], "rb");
    int32_t count, precision, chunk, max_rows;
    if (fread(&count, 4, 1, f) != 1 || fread(&precision, 4, 1, f) != 1) return 2;
    chunk = atoi(argv[3]);
    max_rows = atoi(argv[4]);
    std::vector<scylla_lp> lps(count);
    std::vector<std::vector<int64_t>> rp(count);
    std::vector<std::vector<int32_t>> ci(count);
    std::vector<std::vector<double>> va(count), c(count), b(count), l(count), u(count);
    std::vector<std::vector<char>> s(count);
    for (int q = 0; q < count; ++q) {
        int32_t m, n;
        int64_t nnz;
        if (fread(&m, 4, 1, f) != 1 || fread(&n, 4, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 2;
        rp[q] = rd<int64_t>(f, m + 1);
        ci[q] = rd<int32_t>(f, nnz);
        va[q] = rd<double>(f, nnz);
        c[q] = rd<double>(f, n);
        b[q] = rd<double>(f, m);
        s[q] = rd<char>(f, m);
        l[q] = rd<double>(f, n);
        u[q] = rd<double>(f, n);
        lps[q] = scylla_lp{{m, n, nnz, rp[q].data(), ci[q].data(), va[q].data()}, c[q].data(), b[q].data(),
                           s[q].data(), l[q].data(), u[q].data()};
    }
    fclose(f);
    std::string err;
    for (int q = 0; q < count; ++q) {
        int rc = scy::validate_lp(&lps[q], err);
        if (rc) { printf("invalid %d %s\n", q, err.c_str()); return 3; }
    }
    scy::HostOrient csr, csc;
    int32_t fmt;
    std::vector<int32_t> ro, co;
    if (scy::build_orientations(lps.data(), count, precision, csr, csc, fmt, ro, co, err)) return 4;
    scy::TilePlan pr, pc;
    scy::plan_tiles(csr.ptr, ro, chunk, max_rows, pr);
    scy::plan_tiles(csc.ptr, co, chunk, max_rows, pc);
    FILE *o = fopen(argv[2], "wb");
    std::vector<int32_t> hdr = {fmt, csr.shift, (int32_t)csr.mask, csc.shift, (int32_t)csc.mask, pr.nslots, pc.nslots};
    wr(o, hdr);
    wr(o, ro); wr(o, co);
    for (auto *x : {&csr, &csc}) {
        wr(o, x->ptr); wr(o, x->ent); wr(o, x->v16); wr(o, x->v32); wr(o, x->v64);
    }
    for (auto *p : {&pr, &pc}) {
        wr(o, p->tiles); wr(o, p->longs); wr(o, p->t_begin); wr(o, p->t_end); wr(o, p->l_begin); wr(o, p->l_end);
    }
    const int32_t B = argc > 5 ? atoi(argv[5]) : 0;
    if (B < 0 && argc > 8) {  // direct staged tiles: max_vec group_nnz lanes_min
        for (int d = 0; d < 2; ++d) {
            const scy::HostOrient &x = d == 0 ? csr : csc;
            const std::vector<int32_t> &off = d == 0 ? ro : co, &gof = d == 0 ? co : ro;
            std::vector<uint8_t> dir;
            std::vector<int32_t> tiles;
            scy::plan_direct(x.ptr, off, gof, atoi(argv[6]), atoi(argv[7]), atoi(argv[8]), scy::dpass_k(atoi(argv[8])),
                             dir, tiles);
            std::vector<int32_t> di(dir.begin(), dir.end());
            wr(o, di); wr(o, tiles);
        }
        fclose(o);
        return 0;
    }
    if (B > 0) {
        for (int d = 0; d < 2; ++d) {
            const scy::HostOrient &x = d == 0 ? csr : csc;
            const std::vector<int32_t> &off = d == 0 ? ro : co, &gof = d == 0 ? co : ro;
            scy::BlockedHost bh;
            scy::build_blocked(x, fmt, gof.back(), B, bh);
            scy::BlockedPlan bp;
            scy::plan_blocked(bh, (int32_t)x.ptr.size() - 1, off, chunk, max_rows, bp);
            wr(o, bh.bounds); wr(o, bh.bptr); wr(o, bh.ent); wr(o, bh.v16); wr(o, bh.v32); wr(o, bh.v64);
            wr(o, bp.tiles); wr(o, bp.longs); wr(o, bp.ctiles);
        }
    }
    if (argc > 8) {
        const int32_t max_vec = atoi(argv[6]), sub_chunk = atoi(argv[7]), group_nnz = atoi(argv[8]);
        for (int d = 0; d < 2; ++d) {
            const scy::HostOrient &x = d == 0 ? csr : csc;
            const std::vector<int32_t> &off = d == 0 ? ro : co, &gof = d == 0 ? co : ro;
            scy::StagedPlan sp;
            scy::plan_staged(x.ptr, off, gof, max_vec, sub_chunk, group_nnz, chunk, sp);
            std::vector<int32_t> staged(sp.staged.begin(), sp.staged.end());
            wr(o, sp.tiles); wr(o, sp.sub.tiles); wr(o, sp.sub.longs); wr(o, staged);
            wr(o, sp.rest.tiles); wr(o, sp.rest.longs);
            if (argc > 9) {
                std::vector<uint8_t> cand(sp.staged.size());
                for (size_t q = 0; q < cand.size(); ++q) cand[q] = sp.staged[q] ? 0 : 1;
                scy::SlicedPlan xp;
                scy::plan_sliced(x, fmt, off, gof, cand, max_vec, atoi(argv[9]), sub_chunk, group_nnz, xp);
                std::vector<int32_t> hd = {xp.S, xp.max_slice};
                std::vector<int32_t> sl(xp.sliced.begin(), xp.sliced.end());
                wr(o, hd); wr(o, sl); wr(o, xp.Sq); wr(o, xp.bptr); wr(o, xp.ent); wr(o, xp.tiles); wr(o, xp.sub);
                wr(o, xp.ctiles);
            }
        }
    }
    fclose(o);
    return 0;
}
