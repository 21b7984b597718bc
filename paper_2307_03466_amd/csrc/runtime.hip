// Solver runtime and C ABI of the PDHG library: device-resident batches of
// LPs, device-side preconditioning, tile plans and their autotuner, hipGraph
// capture of one check window (KKT check + decision + R iterations), and
// the host loop that launches windows and polls one status copy per window.
// The pump loop of Algorithm 1 is in pump.hip.
#include "batch.h"

namespace scy {
thread_local std::string g_err;
}  // namespace scy

namespace {

void check_device()
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        throw_err(-ENODEV, "no HIP device visible");
    }
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw_err(-ENODEV, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
}

template <class V>
PassArgs<V> orient_args(scylla_batch *h, OrientRT &o, bool check)
{
    PassArgs<V> p{};
    p.M = o.blocked ? o.bmat : o.mat;
    p.tiles = o.tiles.as<int4>();
    p.ntiles = o.ntiles();
    p.longs = o.longs.as<int4>();
    p.nlong = o.nlong();
    p.st = h->st.as<InstState>();
    p.seg = o.seg.as<V>();
    p.seg64 = o.seg64.as<double>();
    p.part = o.part.as<double>();
    p.lpart = o.lpart.as<double>();
    p.bptr = o.bptr.as<int32_t>();
    p.rows = o.rows;
    p.B = o.blocked ? o.bh.B : 0;
    p.P = o.P.as<V>();
    p.P64 = o.P64.as<double>();
    p.ctiles = o.ctiles.as<int4>();
    p.nctiles = o.blocked ? (int32_t)(o.bplan.ctiles.size() / 4) : 0;
    p.adapt = h->adaptive ? 1 : 0;
    p.ax = h->ax.as<double>();
    p.own_prev = o.row ? h->yp.as<V>() : h->xp.as<V>();
    p.prod_prev = o.row ? h->axp.as<double>() : h->atyp.as<double>();
    if (!o.row && h->has_q) {
        p.q = h->qv.as<V>();
        p.q64 = h->q64.as<double>();
    }
    p.ipart = o.ipart.as<double>();
    p.iplong = o.ipart.as<double>() + 2 * (size_t)o.ipo_long;
    if (h->avg_on && !check) p.avg = o.row ? h->yavg.as<V>() : h->xavg.as<V>();
    if (o.cmp && !check && !o.blocked) {
        p.tiles = o.c_tiles.as<int4>();
        p.ntiles = (int32_t)(o.c_tiles_h.size() / 4);
        p.iplong = o.ipart.as<double>() + 2 * (size_t)o.cipo_long;
    }
    if (o.sliced) {
        p.X = MatView{o.xptr.as<int32_t>(), o.xent.as<uint32_t>(), o.xval.p, o.host.shift, o.host.mask};
        p.xsub = o.xsub.as<int4>();
        p.xS = o.xplan.S;
        p.xSq = o.xsq.as<int32_t>();
        p.xP = o.xP.as<V>();
    }
    if (o.row) {
        p.gvec = check ? h->x.as<V>() : h->xbar.as<V>();
        p.own = h->y.as<V>();
        p.own_ref = h->yr.as<V>();
        p.rhs = h->b_v.as<V>();
        p.diag2 = h->dr2.as<V>();
        p.sense = h->sense.as<uint8_t>();
        p.rhs64 = h->b64.as<double>();
        p.d64 = h->dr64.as<double>();
    } else {
        p.gvec = h->y.as<V>();
        p.own = h->x.as<V>();
        p.bar = h->xbar.as<V>();
        p.own_ref = h->xr.as<V>();
        p.rhs = h->cv.as<V>();
        p.diag2 = h->dc2.as<V>();
        p.lo = h->lv.as<V>();
        p.hi = h->uv.as<V>();
        p.ibnd = h->ibnd.as<V>();
        p.rhs64 = h->c64.as<double>();
        p.lo64 = h->l64.as<double>();
        p.hi64 = h->u64.as<double>();
        p.d64 = h->dc64.as<double>();
    }
    return p;
}

void upload_vals(scylla_batch *h, DevMem &d, const std::vector<uint16_t> &v16, const std::vector<float> &v32,
                 const std::vector<double> &v64)
{
    if (h->fmt == FMT_BF16) upload(d, v16, h->stream);
    else if (h->fmt == FMT_F32) upload(d, v32, h->stream);
    else if (h->fmt == FMT_F64) upload(d, v64, h->stream);
}

// Slot spaces of the adaptive-step partials for the active layout: normal
// tiles then long rows; blocked combine tiles; staged (and sliced) tiles,
// sliced combine tiles, rest tiles, rest long rows.
void ip_layout(OrientRT &o)
{
    auto n4 = [](const std::vector<int32_t> &v) { return (int32_t)(v.size() / 4); };
    o.ipo_long = o.ipo_comb = o.ipo_rest = o.ipo_rlong = 0;
    if (o.staged || o.direct) {
        o.ipo_comb = o.nstiles;
        o.ipo_rest = o.ipo_comb + (o.sliced ? n4(o.xplan.ctiles) : 0);
        o.ipo_rlong = o.ipo_rest + n4(o.splan.rest.tiles);
        o.ip_slots = o.ipo_rlong + n4(o.splan.rest.longs);
    } else if (o.blocked) {
        o.ip_slots = n4(o.bplan.ctiles);
    } else {
        o.ipo_long = n4(o.plan.tiles);
        o.ip_slots = o.ipo_long + n4(o.plan.longs);
    }
    const size_t bytes = 16 * (size_t)std::max(o.ip_slots, 1);
    if (o.ipart.bytes < bytes) o.ipart.alloc(bytes);
}

// Plans the orientation with `ept` nonzeros per thread, normal layout
// (B = 0) or gather-blocked with B blocks, and uploads the plan buffers.
// ept < 0: the tiles of |ept| run by 1024-thread workgroups (kernel choice only)
void set_plan(scylla_batch *h, OrientRT &o, int32_t B, int32_t ept)
{
    const int32_t chunk = 256 * std::abs(ept);
    const std::vector<int32_t> &off = o.row ? h->row_off : h->col_off;
    const size_t vb = (size_t)h->vbytes;
    o.ept = ept;
    o.staged = false;
    o.sliced = false;
    o.direct = false;
    o.cmp = false;
    if (B > 0) {
        if (!o.blocked || o.bh.B != B) {
            build_blocked(o.host, h->fmt, o.gather, B, o.bh);
            upload(o.bptr, o.bh.bptr, h->stream);
            upload(o.bent, o.bh.ent, h->stream);
            upload_vals(h, o.bval, o.bh.v16, o.bh.v32, o.bh.v64);
            HIPC(hipStreamSynchronize(h->stream));
            o.bh.ent.clear();
            o.bh.ent.shrink_to_fit();
            o.bh.v16.clear();
            o.bh.v16.shrink_to_fit();
            o.bh.v32.clear();
            o.bh.v32.shrink_to_fit();
            o.bh.v64.clear();
            o.bh.v64.shrink_to_fit();
            o.bmat = MatView{o.bptr.as<int32_t>(), o.bent.as<uint32_t>(), o.bval.p, o.host.shift, o.host.mask};
            o.P.alloc((size_t)B * std::max(o.rows, 1) * vb);
            o.P64.alloc((size_t)B * std::max(o.rows, 1) * 8);
        }
        o.blocked = true;
        plan_blocked(o.bh, o.rows, off, chunk, 1024, o.bplan);
        upload(o.tiles, o.bplan.tiles, h->stream);
        upload(o.longs, o.bplan.longs, h->stream);
        upload(o.ctiles, o.bplan.ctiles, h->stream);
        o.seg.alloc(std::max<size_t>(1, o.bplan.nslots) * vb);
        o.seg64.alloc(std::max<size_t>(1, o.bplan.nslots) * 8);
        o.part.alloc(std::max<size_t>(1, o.bplan.ctiles.size() / 4) * CHK * 8);
        o.lpart.alloc(8 * CHK);
    } else {
        o.blocked = false;
        plan_tiles(o.host.ptr, off, chunk, 1024, o.plan);
        upload(o.tiles, o.plan.tiles, h->stream);
        upload(o.longs, o.plan.longs, h->stream);
        o.seg.alloc(std::max<size_t>(1, o.plan.nslots) * vb);
        o.seg64.alloc(std::max<size_t>(1, o.plan.nslots) * 8);
        o.part.alloc(std::max<size_t>(1, o.plan.tiles.size() / 4) * CHK * 8);
        o.lpart.alloc(std::max<size_t>(1, o.plan.longs.size() / 4) * CHK * 8);
    }
    ip_layout(o);
    HIPC(hipStreamSynchronize(h->stream));
}

// LDS-staged layout: the normal plan (used by the check) with `ept`, plus
// staged tiles of about `group_nnz` nonzeros for every instance whose
// gathered vector fits in LDS and normal tiles for the others.
void release_sliced(OrientRT &o)
{
    o.sliced = false;
    o.xplan = SlicedPlan();
    o.x_max_vec = o.x_sub = -1;
    o.xptr.release();
    o.xent.release();
    o.xval.release();
    o.xsub.release();
    o.xctiles.release();
    o.xP.release();
    o.xsq.release();
}

// LDS-staged layout; with `slice`, instances too long for LDS (up to 4x)
// are processed in LDS slices (partial sums + row combine) instead of
// normal tiles; with `half`, a workgroup uses at most half the LDS, so two
// workgroups share a CU and overlap one's vector copy with the other's
// gathers (smaller vectors qualify, longer ones take more slices).
void set_staged(scylla_batch *h, OrientRT &o, int32_t ept, int32_t group_nnz, int32_t variant, int32_t slice,
                int32_t half)
{
    set_plan(h, o, 0, ept);
    const std::vector<int32_t> &off = o.row ? h->row_off : h->col_off;
    const std::vector<int32_t> &gofs = o.row ? h->col_off : h->row_off;
    const int32_t chunk = spass_chunk(variant);
    const int32_t max_vec =
        ((half ? h->lds_max / 2 : h->lds_max) - SPASS_STATIC_LDS - LDS_COPY_SLACK) / h->vbytes - chunk;
    plan_staged(o.host.ptr, off, gofs, max_vec, chunk, group_nnz, 256 * std::abs(ept), o.splan);
    std::vector<int32_t> tiles = o.splan.tiles;
    if (slice) {
        if (o.x_max_vec != max_vec || o.x_sub != chunk) {
            std::vector<uint8_t> cand(h->count);
            for (int32_t q = 0; q < h->count; ++q) cand[q] = o.splan.staged[q] ? 0 : 1;
            release_sliced(o);
            build_sliced(o.host, h->fmt, off, gofs, cand, max_vec, 4, chunk, o.xplan);
            o.x_max_vec = max_vec;
            o.x_sub = chunk;
            if (o.xplan.S > 0) {
                upload(o.xsq, o.xplan.Sq, h->stream);
                upload(o.xptr, o.xplan.bptr, h->stream);
                upload(o.xent, o.xplan.ent, h->stream);
                upload_vals(h, o.xval, o.xplan.v16, o.xplan.v32, o.xplan.v64);
                o.xP.alloc((size_t)o.xplan.S * std::max(o.rows, 1) * h->vbytes);
                HIPC(hipStreamSynchronize(h->stream));
                o.xplan.ent.clear();
                o.xplan.ent.shrink_to_fit();
                o.xplan.v16.clear();
                o.xplan.v16.shrink_to_fit();
                o.xplan.v32.clear();
                o.xplan.v32.shrink_to_fit();
                o.xplan.v64.clear();
                o.xplan.v64.shrink_to_fit();
            }
        }
        o.sliced = o.xplan.S > 0;
    } else {
        o.sliced = false;
    }
    if (o.sliced) {
        tile_sliced(off, o.rows, chunk, group_nnz, o.xplan);
        upload(o.xsub, o.xplan.sub, h->stream);
        upload(o.xctiles, o.xplan.ctiles, h->stream);
        tiles.insert(tiles.end(), o.xplan.tiles.begin(), o.xplan.tiles.end());
        // normal tiles only for instances neither staged nor sliced
        std::vector<uint8_t> skip(h->count);
        for (int32_t q = 0; q < h->count; ++q) skip[q] = (o.splan.staged[q] || o.xplan.sliced[q]) ? 1 : 0;
        plan_tiles(o.host.ptr, off, 256 * std::abs(ept), 1024, o.splan.rest, skip.data());
    }
    upload(o.stiles, tiles, h->stream);
    o.stiles_h = tiles;
    upload(o.subtiles, o.splan.sub.tiles, h->stream);
    upload(o.gofs, gofs, h->stream);
    upload(o.rtiles, o.splan.rest.tiles, h->stream);
    upload(o.rlongs, o.splan.rest.longs, h->stream);
    o.rseg.alloc(std::max<size_t>(1, o.splan.rest.nslots) * h->vbytes);
    const int32_t vec = std::max({o.splan.max_vec, o.sliced ? o.xplan.max_slice : 0, 1});
    o.shmem = (size_t)(chunk + vec) * h->vbytes + LDS_COPY_SLACK;
    PassArgs<float> pf{};
    PassArgs<double> pd{};
    if (h->vbytes == 4)
        for (int c : {0, (int)FMT_CACHED})  // both matrix load policies
            launch_staged<float>(pf, h->fmt | c, o.row ? DIR_ROW : DIR_COL, variant, 0, o.shmem, h->stream, true);
    else
        launch_staged<double>(pd, h->fmt, o.row ? DIR_ROW : DIR_COL, variant, 0, o.shmem, h->stream, true);
    HIPC(hipStreamSynchronize(h->stream));
    o.nstiles = (int32_t)(tiles.size() / 4);
    o.staged = o.nstiles > 0;
    o.staged_nnz = group_nnz;
    o.svariant = variant;
    o.shalf = half != 0;
    ip_layout(o);
}

// Direct staged layout: instances whose whole gathered vector fits in the
// LDS get direct tiles of about `group_nnz` nonzeros (at least `lanes_min`
// lanes per row), the others normal tiles with `ept`.
void set_direct(scylla_batch *h, OrientRT &o, int32_t ept, int32_t group_nnz, int32_t lanes_min)
{
    set_plan(h, o, 0, ept);
    const std::vector<int32_t> &off = o.row ? h->row_off : h->col_off;
    const std::vector<int32_t> &gofs = o.row ? h->col_off : h->row_off;
    // room for the kernel's static LDS and the copy's alignment slack
    const int32_t max_vec = (h->lds_max - 1024 - LDS_COPY_SLACK) / h->vbytes;
    const int32_t k = dpass_k(lanes_min);
    plan_direct(o.host.ptr, off, gofs, max_vec, group_nnz, lanes_min, k, o.dinst, o.dtiles_h);
    upload(o.dtiles, o.dtiles_h, h->stream);
    plan_tiles(o.host.ptr, off, 256 * std::abs(ept), 1024, o.splan.rest, o.dinst.data());
    upload(o.gofs, gofs, h->stream);
    upload(o.rtiles, o.splan.rest.tiles, h->stream);
    upload(o.rlongs, o.splan.rest.longs, h->stream);
    o.rseg.alloc(std::max<size_t>(1, o.splan.rest.nslots) * h->vbytes);
    int32_t vmax = 1;
    for (int32_t q = 0; q < h->count; ++q)
        if (o.dinst[q]) vmax = std::max(vmax, gofs[q + 1] - gofs[q]);
    o.dshmem = (size_t)vmax * h->vbytes + LDS_COPY_SLACK;
    PassArgs<float> pf{};
    PassArgs<double> pd{};
    if (h->vbytes == 4)
        for (int c : {0, (int)FMT_CACHED})  // both matrix load policies
            launch_direct<float>(pf, h->fmt | c, o.row ? DIR_ROW : DIR_COL, k, 0, o.dshmem, h->stream, true);
    else launch_direct<double>(pd, h->fmt, o.row ? DIR_ROW : DIR_COL, k, 0, o.dshmem, h->stream, true);
    HIPC(hipStreamSynchronize(h->stream));
    o.nstiles = (int32_t)(o.dtiles_h.size() / 4);
    o.direct = o.nstiles > 0;
    o.dnnz = group_nnz;
    o.dlanes = lanes_min;
    ip_layout(o);
}

// Drops the blocked layout's device copy (after the tuner chose normal).
void drop_blocked(OrientRT &o)
{
    o.bptr.release();
    o.bent.release();
    o.bval.release();
    o.P.release();
    o.P64.release();
    o.ctiles.release();
    o.bh = BlockedHost();
    o.bplan = BlockedPlan();
}

void refresh_info(scylla_batch *h)
{
    h->hinfo.resize(h->count);
    for (int32_t q = 0; q < h->count; ++q) {
        InstInfo &I = h->hinfo[q];
        I.row0 = h->row_off[q];
        I.row1 = h->row_off[q + 1];
        I.col0 = h->col_off[q];
        I.col1 = h->col_off[q + 1];
        for (int d = 0; d < 2; ++d) {
            OrientRT &o = d == 0 ? h->orow : h->ocol;
            int32_t t0, t1, l0 = 0, l1 = 0;
            if (o.blocked) {
                t0 = o.bplan.ct_begin[q];
                t1 = o.bplan.ct_end[q];
            } else {
                t0 = o.plan.t_begin[q];
                t1 = o.plan.t_end[q];
                l0 = o.plan.l_begin[q];
                l1 = o.plan.l_end[q];
            }
            if (d == 0) {
                I.rt0 = t0; I.rt1 = t1; I.lr0 = l0; I.lr1 = l1;
            } else {
                I.ct0 = t0; I.ct1 = t1; I.lc0 = l0; I.lc1 = l1;
            }
            // slots of this instance's epilogues in the iteration partials
            int32_t (*ir)[2] = I.ir[d];
            for (int r = 0; r < 3; ++r) ir[r][0] = ir[r][1] = 0;
            if (o.direct) {
                if (o.dinst[q]) {
                    int32_t a = -1, b = -1;
                    for (size_t t = 0; t < o.dtiles_h.size() / 4; ++t)
                        if (o.dtiles_h[4 * t + 2] == q) {
                            if (a < 0) a = (int32_t)t;
                            b = (int32_t)t + 1;
                        }
                    if (a >= 0) { ir[0][0] = a; ir[0][1] = b; }
                } else {
                    ir[0][0] = o.ipo_rest + o.splan.rest.t_begin[q];
                    ir[0][1] = o.ipo_rest + o.splan.rest.t_end[q];
                    ir[1][0] = o.ipo_rlong + o.splan.rest.l_begin[q];
                    ir[1][1] = o.ipo_rlong + o.splan.rest.l_end[q];
                }
            } else if (o.staged) {
                if (o.splan.staged[q]) {
                    int32_t a = -1, b = -1;
                    for (size_t t = 0; t < o.splan.tiles.size() / 4; ++t)
                        if (o.splan.tiles[4 * t + 2] == q) {
                            if (a < 0) a = (int32_t)t;
                            b = (int32_t)t + 1;
                        }
                    if (a >= 0) { ir[0][0] = a; ir[0][1] = b; }
                } else if (o.sliced && o.xplan.sliced[q]) {
                    int32_t a = -1, b = -1;
                    for (size_t t = 0; t < o.xplan.ctiles.size() / 4; ++t)
                        if (o.xplan.ctiles[4 * t + 2] == q) {
                            if (a < 0) a = (int32_t)t;
                            b = (int32_t)t + 1;
                        }
                    if (a >= 0) { ir[0][0] = o.ipo_comb + a; ir[0][1] = o.ipo_comb + b; }
                } else {
                    ir[0][0] = o.ipo_rest + o.splan.rest.t_begin[q];
                    ir[0][1] = o.ipo_rest + o.splan.rest.t_end[q];
                    ir[1][0] = o.ipo_rlong + o.splan.rest.l_begin[q];
                    ir[1][1] = o.ipo_rlong + o.splan.rest.l_end[q];
                }
            } else if (o.blocked) {
                ir[0][0] = o.bplan.ct_begin[q];
                ir[0][1] = o.bplan.ct_end[q];
            } else {
                ir[0][0] = o.plan.t_begin[q];
                ir[0][1] = o.plan.t_end[q];
                ir[1][0] = o.ipo_long + o.plan.l_begin[q];
                ir[1][1] = o.ipo_long + o.plan.l_end[q];
            }
        }
    }
    upload(h->info, h->hinfo, h->stream);
    HIPC(hipStreamSynchronize(h->stream));
}

void invalidate_graph(scylla_batch *h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->graph_R = 0;
}

template <class V>
void launch_orient(scylla_batch *h, OrientRT &o, const PassArgs<V> &p, int jw, bool check, hipStream_t s)
{
    const int dir = o.row ? DIR_ROW : DIR_COL;
    // the iteration passes read the matrix with the orientation's load
    // policy (the checks, once per window, stream it)
    const int ifmt = h->fmt | (o.cached && h->vbytes == 4 ? (int)FMT_CACHED : 0);
    // iteration launches take the compacted tile lists when there are any
    const bool cmp = o.cmp && !check;
    auto n4 = [](const std::vector<int32_t> &v) { return (int32_t)(v.size() / 4); };
    if (o.direct && !check) {
        PassArgs<V> pd = p;
        pd.dtiles = cmp ? o.c_dtiles.as<int4>() : o.dtiles.as<int4>();
        pd.ndtiles = cmp ? n4(o.c_dtiles_h) : o.nstiles;
        pd.gofs = o.gofs.as<int32_t>();
        PassArgs<V> pr = p;  // normal tiles of the other instances
        pr.tiles = cmp ? o.c_rtiles.as<int4>() : o.rtiles.as<int4>();
        pr.ntiles = cmp ? n4(o.c_rtiles_h) : n4(o.splan.rest.tiles);
        pr.longs = o.rlongs.as<int4>();
        pr.nlong = (int32_t)(o.splan.rest.longs.size() / 4);
        pr.seg = o.rseg.as<V>();
        pr.ipart = o.ipart.as<double>() + 2 * (size_t)(cmp ? o.cipo_rest : o.ipo_rest);
        pr.iplong = o.ipart.as<double>() + 2 * (size_t)(cmp ? o.cipo_rlong : o.ipo_rlong);
        const bool fork = pr.ntiles > 0 || pr.nlong > 0;
        if (fork) {
            HIPC(hipEventRecord(h->fork, s));
            HIPC(hipStreamWaitEvent(h->side, h->fork, 0));
            launch_pass<V>(pr, ifmt, dir, o.ept, jw, false, false, h->side);
            HIPC(hipEventRecord(h->join, h->side));
        }
        launch_direct<V>(pd, ifmt, dir, dpass_k(o.dlanes), jw, o.dshmem, s, false);
        if (fork) HIPC(hipStreamWaitEvent(s, h->join, 0));
        return;
    }
    if (o.staged && !check) {
        PassArgs<V> ps = p;
        ps.tiles = cmp ? o.c_stiles.as<int4>() : o.stiles.as<int4>();
        ps.ntiles = cmp ? n4(o.c_stiles_h) : o.nstiles;
        ps.gofs = o.gofs.as<int32_t>();
        ps.sub = o.subtiles.as<int4>();
        PassArgs<V> pc = ps;  // row combine of the sliced instances
        if (o.sliced) {
            pc.ctiles = cmp ? o.c_xctiles.as<int4>() : o.xctiles.as<int4>();
            pc.nctiles = cmp ? n4(o.c_xctiles_h) : n4(o.xplan.ctiles);
            pc.B = o.xplan.S;
            pc.bq = o.xsq.as<int32_t>();
            pc.P = o.xP.as<V>();
            pc.ipart = o.ipart.as<double>() + 2 * (size_t)(cmp ? o.cipo_comb : o.ipo_comb);
        }
        PassArgs<V> pr = p;
        pr.tiles = cmp ? o.c_rtiles.as<int4>() : o.rtiles.as<int4>();
        pr.ntiles = cmp ? n4(o.c_rtiles_h) : n4(o.splan.rest.tiles);
        pr.longs = o.rlongs.as<int4>();
        pr.nlong = (int32_t)(o.splan.rest.longs.size() / 4);
        pr.seg = o.rseg.as<V>();
        pr.ipart = o.ipart.as<double>() + 2 * (size_t)(cmp ? o.cipo_rest : o.ipo_rest);
        pr.iplong = o.ipart.as<double>() + 2 * (size_t)(cmp ? o.cipo_rlong : o.ipo_rlong);
        const bool fork = pr.ntiles > 0 || pr.nlong > 0;
        // the kinds of tiles touch disjoint instances: run the normal tiles
        // as a second branch (fork on s, side stream, join)
        if (fork) {
            HIPC(hipEventRecord(h->fork, s));
            HIPC(hipStreamWaitEvent(h->side, h->fork, 0));
            launch_pass<V>(pr, ifmt, dir, o.ept, jw, false, false, h->side);
            HIPC(hipEventRecord(h->join, h->side));
        }
        launch_staged<V>(ps, ifmt, dir, o.svariant, jw, o.shmem, s, false);
        if (o.sliced) launch_combine<V>(pc, dir, jw, s);
        if (fork) HIPC(hipStreamWaitEvent(s, h->join, 0));
        return;
    }
    launch_pass<V>(p, ifmt, dir, o.ept, jw, check, o.blocked, s);
}

template <class V>
TinyArgs<V> tiny_args(scylla_batch *h)
{
    TinyArgs<V> a{};
    a.R = h->orow.mat;
    a.C = h->ocol.mat;
    a.x = h->x.as<V>();
    a.xbar = h->xbar.as<V>();
    a.xr = h->xr.as<V>();
    a.y = h->y.as<V>();
    a.yr = h->yr.as<V>();
    a.c = h->cv.as<V>();
    a.l = h->lv.as<V>();
    a.u = h->uv.as<V>();
    a.dc2 = h->dc2.as<V>();
    a.b = h->b_v.as<V>();
    a.dr2 = h->dr2.as<V>();
    a.sense = h->sense.as<uint8_t>();
    a.c64 = h->c64.as<double>();
    a.l64 = h->l64.as<double>();
    a.u64 = h->u64.as<double>();
    a.b64 = h->b64.as<double>();
    a.dr64 = h->dr64.as<double>();
    a.dc64 = h->dc64.as<double>();
    a.st = h->st.as<InstState>();
    a.info = h->info.as<InstInfo>();
    a.adapt = h->adaptive ? 1 : 0;
    a.xp = h->xp.as<V>();
    a.yp = h->yp.as<V>();
    a.axp = h->axp.as<double>();
    a.atyp = h->atyp.as<double>();
    if (h->has_q) {
        a.q = h->qv.as<V>();
        a.q64 = h->q64.as<double>();
    }
    return a;
}

template <class V>
void enqueue_window(scylla_batch *h, int32_t R, bool tiny, hipStream_t s)
{
    if (tiny) {
        launch_tiny<V>(tiny_args<V>(h), h->fmt, h->count, R, h->tiny_shmem, s, false);
        return;
    }
    const PassArgs<V> rc = orient_args<V>(h, h->orow, true), cc = orient_args<V>(h, h->ocol, true);
    launch_orient<V>(h, h->orow, rc, 0, true, s);
    launch_orient<V>(h, h->ocol, cc, 0, true, s);
    DecideArgs d{h->st.as<InstState>(), h->info.as<InstInfo>(), h->orow.part.as<double>(),
                 h->orow.lpart.as<double>(), h->ocol.part.as<double>(), h->ocol.lpart.as<double>(), R};
    if (h->avg_on) {
        // the same check of the running average (x_avg, y_avg), into its own
        // partials, without the infeasibility terms
        PassArgs<V> ra = rc, ca = cc;
        ra.gvec = h->xavg.as<V>();
        ra.own = h->yavg.as<V>();
        ca.gvec = h->yavg.as<V>();
        ca.own = h->xavg.as<V>();
        for (PassArgs<V> *a : {&ra, &ca}) {
            a->own_prev = nullptr;
            a->prod_prev = nullptr;
            a->ax = h->adaptive ? h->axavg.as<double>() : nullptr;
        }
        ra.part = h->orow.part2.as<double>();
        ra.lpart = h->orow.lpart2.as<double>();
        ca.part = h->ocol.part2.as<double>();
        ca.lpart = h->ocol.lpart2.as<double>();
        launch_orient<V>(h, h->orow, ra, 0, true, s);
        launch_orient<V>(h, h->ocol, ca, 0, true, s);
        d.rpart2 = ra.part;
        d.lrpart2 = ra.lpart;
        d.cpart2 = ca.part;
        d.lcpart2 = ca.lpart;
    }
    launch_decide(d, h->count, s);
    if (h->avg_on)
        launch_take_avg<V>(h->st.as<InstState>(), h->info.as<InstInfo>(), h->x.as<V>(), h->y.as<V>(),
                           h->xavg.as<V>(), h->yavg.as<V>(), h->adaptive ? h->ax.as<double>() : nullptr,
                           h->adaptive ? h->axavg.as<double>() : nullptr, h->count, s);
    const PassArgs<V> ri = orient_args<V>(h, h->orow, false), ci = orient_args<V>(h, h->ocol, false);
    for (int32_t j = 0; j < R; ++j) {
        launch_orient<V>(h, h->ocol, ci, j, false, s);
        launch_orient<V>(h, h->orow, ri, j, false, s);
        if (h->adaptive) {
            const StepArgs a{h->st.as<InstState>(), h->info.as<InstInfo>(), h->orow.ipart.as<double>(),
                             h->ocol.ipart.as<double>(), j};
            launch_step(a, h->count, s);
        }
    }
}

// Captures and instantiates one check window of R iterations with the
// current tile lists.
hipGraphExec_t capture_window(scylla_batch *h, int32_t R, bool tiny)
{
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    HIPC(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    if (h->vbytes == 4) enqueue_window<float>(h, R, tiny, h->cap);
    else enqueue_window<double>(h, R, tiny, h->cap);
    HIPC(hipStreamEndCapture(h->cap, &g));
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPC(e);
    return ex;
}

void ensure_graph(scylla_batch *h, int32_t R, bool tiny)
{
    if (h->gexec && h->graph_R == R && h->graph_tiny == tiny && h->graph_adapt == h->adaptive &&
        h->graph_avg == h->avg_on)
        return;
    invalidate_graph(h);
    if (h->avg_on && !tiny) {
        // partials of the running average's check (allocated before capture)
        for (OrientRT *o : {&h->orow, &h->ocol}) {
            if (o->part2.bytes < o->part.bytes) o->part2.alloc(o->part.bytes);
            if (o->lpart2.bytes < o->lpart.bytes) o->lpart2.alloc(o->lpart.bytes);
        }
    }
    h->gexec = capture_window(h, R, tiny);
    h->graph_R = R;
    h->graph_tiny = tiny;
    h->graph_adapt = h->adaptive;
    h->graph_avg = h->avg_on;
}

// ---- finished instances out of the iteration launches
//
// A finished instance's workgroups still start, read their tile and the
// instance state, and exit; late in a batched solve that costs more than
// the running instances' work.  When the tiles of the running instances
// fall to half of those the window graph launches, the tile lists of the
// iteration launches are cut to the running instances (in their order, so
// every result is unchanged bit for bit), the adaptive-step slot ranges are
// renumbered to match, and a window graph over the cut lists takes over.
// The copies are ordered on the stream behind the windows in flight; an
// instance that stops never runs again within a solve, so lists cut from an
// earlier state hold every tile that can still run.  The check launches
// keep the full lists (once per window).  Gather-blocked orientations (one
// large instance) are not cut.

// Tiles of the iteration launches of o: all (run = NULL), or those of the
// instances with run[q] set.
static int64_t iter_tiles(const OrientRT &o, const uint8_t *run)
{
    if (o.blocked) return 0;
    auto cnt = [&](const std::vector<int32_t> &t) {
        int64_t n = 0;
        for (size_t i = 2; i < t.size(); i += 4) n += (!run || run[t[i] & 0xffffff]) ? 1 : 0;
        return n;
    };
    if (o.direct) return cnt(o.dtiles_h) + cnt(o.splan.rest.tiles);
    if (o.staged) return cnt(o.stiles_h) + (o.sliced ? cnt(o.xplan.ctiles) : 0) + cnt(o.splan.rest.tiles);
    return cnt(o.plan.tiles);
}

// The tiles (4 ints, instance in the low 24 bits of the third) of the
// instances with run[q] set, in order; [a[q], b[q]) is instance q's range
// in the kept list (empty when it has none).
static void keep_tiles(const std::vector<int32_t> &t, const uint8_t *run, std::vector<int32_t> &out,
                       std::vector<int32_t> &a, std::vector<int32_t> &b)
{
    out.clear();
    std::fill(a.begin(), a.end(), -1);
    std::fill(b.begin(), b.end(), 0);
    for (size_t i = 0; i + 3 < t.size(); i += 4) {
        const int32_t q = t[i + 2] & 0xffffff;
        if (!run[q]) continue;
        const int32_t k = (int32_t)(out.size() / 4);
        if (a[q] < 0) a[q] = k;
        b[q] = k + 1;
        out.insert(out.end(), t.begin() + i, t.begin() + i + 4);
    }
    for (size_t q = 0; q < a.size(); ++q)
        if (a[q] < 0) a[q] = 0;
}

// Cuts the iteration lists of orientation d and writes its slot ranges into
// h->hinfo_c (which starts as a copy of h->hinfo).
static void cut_orient(scylla_batch *h, OrientRT &o, int d, const uint8_t *run)
{
    if (o.blocked) return;
    const int32_t count = h->count;
    auto n4 = [](const std::vector<int32_t> &v) { return (int32_t)(v.size() / 4); };
    std::vector<int32_t> a1(count), b1(count), a2(count), b2(count), a3(count), b3(count);
    o.c_tiles_h.clear();
    o.c_stiles_h.clear();
    o.c_xctiles_h.clear();
    o.c_rtiles_h.clear();
    o.c_dtiles_h.clear();
    if (o.direct) {
        keep_tiles(o.dtiles_h, run, o.c_dtiles_h, a1, b1);
        keep_tiles(o.splan.rest.tiles, run, o.c_rtiles_h, a3, b3);
        o.cipo_comb = o.cipo_rest = n4(o.c_dtiles_h);
        o.cipo_rlong = o.cipo_rest + n4(o.c_rtiles_h);
    } else if (o.staged) {
        keep_tiles(o.stiles_h, run, o.c_stiles_h, a1, b1);
        if (o.sliced) keep_tiles(o.xplan.ctiles, run, o.c_xctiles_h, a2, b2);
        keep_tiles(o.splan.rest.tiles, run, o.c_rtiles_h, a3, b3);
        o.cipo_comb = n4(o.c_stiles_h);
        o.cipo_rest = o.cipo_comb + n4(o.c_xctiles_h);
        o.cipo_rlong = o.cipo_rest + n4(o.c_rtiles_h);
    } else {
        keep_tiles(o.plan.tiles, run, o.c_tiles_h, a1, b1);
        o.cipo_long = n4(o.c_tiles_h);
    }
    for (int32_t q = 0; q < count; ++q) {
        int32_t (*ir)[2] = h->hinfo_c[q].ir[d];
        for (int r = 0; r < 3; ++r) ir[r][0] = ir[r][1] = 0;
        if (!run[q]) continue;
        auto rest = [&]() {
            ir[0][0] = o.cipo_rest + a3[q];
            ir[0][1] = o.cipo_rest + b3[q];
            ir[1][0] = o.cipo_rlong + o.splan.rest.l_begin[q];
            ir[1][1] = o.cipo_rlong + o.splan.rest.l_end[q];
        };
        if (o.direct) {
            if (o.dinst[q]) {
                ir[0][0] = a1[q];
                ir[0][1] = b1[q];
            } else {
                rest();
            }
        } else if (o.staged) {
            if (o.splan.staged[q]) {
                ir[0][0] = a1[q];
                ir[0][1] = b1[q];
            } else if (o.sliced && o.xplan.sliced[q]) {
                ir[0][0] = o.cipo_comb + a2[q];
                ir[0][1] = o.cipo_comb + b2[q];
            } else {
                rest();
            }
        } else {
            ir[0][0] = a1[q];
            ir[0][1] = b1[q];
            ir[1][0] = o.cipo_long + o.plan.l_begin[q];
            ir[1][1] = o.cipo_long + o.plan.l_end[q];
        }
    }
    o.cmp = true;
}

// Device lists and pinned staging for cutting, sized for the full lists
// (called with the stream idle, before the solve's first window).
static void prepare_cut(scylla_batch *h)
{
    size_t ints = 0;
    auto need = [&](DevMem &d, const std::vector<int32_t> &full) {
        const size_t b = std::max<size_t>(full.size(), 4) * 4;
        if (d.bytes < b) d.alloc(b);
        ints += full.size();
    };
    for (OrientRT *o : {&h->orow, &h->ocol}) {
        if (o->blocked) continue;
        if (o->direct) {
            need(o->c_dtiles, o->dtiles_h);
            need(o->c_rtiles, o->splan.rest.tiles);
        } else if (o->staged) {
            need(o->c_stiles, o->stiles_h);
            if (o->sliced) need(o->c_xctiles, o->xplan.ctiles);
            need(o->c_rtiles, o->splan.rest.tiles);
        } else {
            need(o->c_tiles, o->plan.tiles);
        }
    }
    const size_t bytes = ints * 4 + sizeof(InstInfo) * (size_t)h->count;
    if (h->cstage_bytes < bytes) {
        if (h->cstage) (void)hipHostFree(h->cstage);
        h->cstage = nullptr;
        h->cstage_bytes = 0;
        HIPC(hipHostMalloc(&h->cstage, bytes, hipHostMallocDefault));
        h->cstage_bytes = bytes;
    }
}

// Cuts both orientations to the instances with run[q] set and queues the
// copies of the cut lists and slot ranges on the stream.  The staging
// buffer is reused: the caller cuts again only after a window launched
// behind these copies has completed.
static void cut_lists(scylla_batch *h, const uint8_t *run)
{
    h->hinfo_c = h->hinfo;
    cut_orient(h, h->orow, 0, run);
    cut_orient(h, h->ocol, 1, run);
    char *st = static_cast<char *>(h->cstage);
    auto put = [&](void *dst, const void *src, size_t bytes) {
        if (bytes == 0) return;
        memcpy(st, src, bytes);
        HIPC(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, h->stream));
        st += bytes;
    };
    for (OrientRT *o : {&h->orow, &h->ocol}) {
        if (!o->cmp) continue;
        put(o->c_tiles.p, o->c_tiles_h.data(), o->c_tiles_h.size() * 4);
        put(o->c_stiles.p, o->c_stiles_h.data(), o->c_stiles_h.size() * 4);
        put(o->c_xctiles.p, o->c_xctiles_h.data(), o->c_xctiles_h.size() * 4);
        put(o->c_rtiles.p, o->c_rtiles_h.data(), o->c_rtiles_h.size() * 4);
        put(o->c_dtiles.p, o->c_dtiles_h.data(), o->c_dtiles_h.size() * 4);
    }
    put(h->info.p, h->hinfo_c.data(), sizeof(InstInfo) * (size_t)h->count);
}

// Back to the full lists (stream drained first); safe to call at any time.
static void uncut(scylla_batch *h) noexcept
{
    const bool any = h->cexec || !h->retired.empty() || h->orow.cmp || h->ocol.cmp;
    if (!any) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->cexec) (void)hipGraphExecDestroy(h->cexec);
    h->cexec = nullptr;
    for (hipGraphExec_t g : h->retired) (void)hipGraphExecDestroy(g);
    h->retired.clear();
    h->orow.cmp = h->ocol.cmp = false;
    if (!h->hinfo.empty() && h->info.p) {
        (void)hipMemcpyAsync(h->info.p, h->hinfo.data(), sizeof(InstInfo) * h->hinfo.size(), hipMemcpyHostToDevice,
                             h->stream);
        (void)hipStreamSynchronize(h->stream);
    }
}

// Scratch outputs and an always-running state so a pass can be launched on
// its own without changing the iterates (autotuning and pass timing).  The
// gathered vectors are the real ones, so cache behaviour is representative.
template <class V>
struct PassTimer {
    DevMem trial_st, sx, sbar, sy;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    scylla_batch *h;
    explicit PassTimer(scylla_batch *hh) : h(hh)
    {
        std::vector<InstState> ts(h->count);
        for (auto &S : ts) {
            memset(&S, 0, sizeof(S));
            S.status = ST_RUN;
            S.nrun = 1 << 30;
        }
        upload(trial_st, ts, h->stream);
        sx.alloc((size_t)std::max(h->N, 1) * sizeof(V));
        sbar.alloc((size_t)std::max(h->N, 1) * sizeof(V));
        sy.alloc((size_t)std::max(h->M, 1) * sizeof(V));
        HIPC(hipMemsetAsync(sx.p, 0, sx.bytes, h->stream));
        HIPC(hipMemsetAsync(sbar.p, 0, sbar.bytes, h->stream));
        HIPC(hipMemsetAsync(sy.p, 0, sy.bytes, h->stream));
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        HIPC(hipStreamSynchronize(h->stream));
    }
    ~PassTimer()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    // average milliseconds of one pass (all its launches) of orientation o,
    // alone or (paired) together with one pass of the other orientation in
    // its current layout.  The tuner times candidates paired, where they
    // run: a pass timed alone finds the caches as it left them, and on the
    // pump batch a candidate 5 % faster alone made the iteration slower.
    double time(OrientRT &o, int reps, bool paired = true)
    {
        OrientRT &w = o.row ? h->ocol : h->orow;
        PassArgs<V> p = orient_args<V>(h, o, false), q = orient_args<V>(h, w, false);
        for (PassArgs<V> *a : {&p, &q}) {
            a->st = trial_st.as<InstState>();
            a->bar = sbar.as<V>();
            a->avg = nullptr;
        }
        p.own = o.row ? sy.as<V>() : sx.as<V>();
        q.own = w.row ? sy.as<V>() : sx.as<V>();
        if (paired) launch_orient<V>(h, w, q, 1, false, h->stream);
        launch_orient<V>(h, o, p, 1, false, h->stream);
        HIPC(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) {
            if (paired) launch_orient<V>(h, w, q, 1, false, h->stream);
            launch_orient<V>(h, o, p, 1, false, h->stream);
        }
        HIPC(hipEventRecord(e1, h->stream));
        HIPC(hipEventSynchronize(e1));
        HIPC(hipGetLastError());
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms / reps;
    }
};

// ------------------------------------------------------------ tuning cache
// Layout choices per (device arch, precision, format, shape) so handles of
// the same shape skip the timing runs.  Kept per process; when the
// environment variable SCYLLA_TUNE_CACHE names a file, entries are read from
// it once and new ones appended (one line: key and 8 integers).
struct TuneChoice {
    int32_t v[8];  // row: mode(B, -1 staged), ept, staged nnz, variant; col: same
};

std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;

std::string tune_key(scylla_batch *h)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    // shape hash: sizes, instance offsets and log2 row-length histograms
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        hsh ^= v;
        hsh *= 1099511628211ull;
    };
    mix((uint64_t)h->count);
    mix((uint64_t)h->M);
    mix((uint64_t)h->N);
    mix((uint64_t)h->NNZ);
    for (int32_t q = 0; q <= h->count; ++q) {
        mix((uint64_t)h->row_off[q]);
        mix((uint64_t)h->col_off[q]);
    }
    for (int d = 0; d < 2; ++d) {
        const std::vector<int32_t> &ptr = d == 0 ? h->orow.host.ptr : h->ocol.host.ptr;
        uint64_t hist[33] = {0};
        for (size_t i = 0; i + 1 < ptr.size(); ++i) {
            int32_t len = ptr[i + 1] - ptr[i], b = 0;
            while (len > 0) {
                len >>= 1;
                ++b;
            }
            hist[b]++;
        }
        for (uint64_t c : hist) mix(c);
    }
    std::ostringstream os;
    os << arch << ":p" << h->precision << ":f" << h->fmt << ":" << std::hex << hsh;
    return os.str();
}

bool tune_lookup(const std::string &key, TuneChoice &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const char *path = getenv("SCYLLA_TUNE_CACHE");
    if (!g_tune_loaded && path) {
        std::ifstream f(path);
        std::string k;
        TuneChoice c;
        while (f >> k >> c.v[0] >> c.v[1] >> c.v[2] >> c.v[3] >> c.v[4] >> c.v[5] >> c.v[6] >> c.v[7]) g_tune[k] = c;
    }
    g_tune_loaded = true;
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneChoice &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = c;
    if (const char *path = getenv("SCYLLA_TUNE_CACHE")) {
        std::ofstream f(path, std::ios::app);
        f << key;
        for (int i = 0; i < 8; ++i) f << ' ' << c.v[i];
        f << '\n';
    }
}

void apply_choice(scylla_batch *h, OrientRT &o, const int32_t *v)
{
    const int32_t v3 = v[3] & ~64;  // bit 64: plain (cacheable) matrix loads
    if (v[0] == -2) {
        set_direct(h, o, v[1], v[2], v3);
        drop_blocked(o);
        release_sliced(o);
    } else if (v[0] < 0) {
        set_staged(h, o, v[1], v[2], v3 & 3, (v3 >> 2) & 1, (v3 >> 3) & 1);
        drop_blocked(o);
    } else {
        set_plan(h, o, v[0], v[1]);
        if (v[0] == 0) drop_blocked(o);
    }
    o.cached = (v[3] & 64) != 0 && h->vbytes == 4;
}

TuneChoice current_choice(scylla_batch *h)
{
    TuneChoice c;
    for (int d = 0; d < 2; ++d) {
        const OrientRT &o = d == 0 ? h->orow : h->ocol;
        int32_t *v = c.v + 4 * d;
        v[0] = o.direct ? -2 : (o.staged ? -1 : (o.blocked ? o.bh.B : 0));
        v[1] = o.ept;
        v[2] = o.direct ? o.dnnz : (o.staged ? o.staged_nnz : 0);
        v[3] = o.direct ? o.dlanes
                        : (o.staged ? (o.svariant | (o.sliced ? 4 : 0) | (o.shalf ? 8 : 0)) : 0);
        if (o.cached) v[3] |= 64;
    }
    return c;
}

// Times the layout / tile-size candidates of each orientation and keeps the
// fastest: the normal layout with 2, 4, 8 or 16 nonzeros per thread, and, when
// the gathered vector is larger than 2 MB, the gather-blocked layout with 2,
// 4 or 8 blocks (one block per XCD, per XCD pair or per four XCDs).
template <class V>
void autotune(scylla_batch *h)
{
    const std::string key = tune_key(h);
    TuneChoice cached;
    if (tune_lookup(key, cached)) {
        apply_choice(h, h->orow, cached.v);
        apply_choice(h, h->ocol, cached.v + 4);
        refresh_info(h);
        invalidate_graph(h);
        h->tuned = true;
        return;
    }
    const int epts[6] = {2, 4, 8, 16, -8, -16};
    // The matrix load policy first, on the initial layout (both passes
    // timed together): whether an iteration's data fits the device's
    // last-level cache hardly depends on the layout, and the layouts are
    // then ranked under the policy they will run with; the policy is timed
    // again on the chosen layouts at the end.
    h->orow.cached = h->ocol.cached = false;
    // SCYLLA_TUNE_TRACE=1: one line per candidate on stderr (plan time on
    // the host, measured pass time)
    const bool trace = getenv("SCYLLA_TUNE_TRACE") != nullptr;
    PassTimer<V> timer(h);
    if (h->vbytes == 4) {
        const double t_nt = timer.time(h->orow, 20);
        h->orow.cached = h->ocol.cached = true;
        const double t_c = timer.time(h->orow, 20);
        if (trace) fprintf(stderr, "tune load policy first: non-temporal %.3f ms, cached %.3f ms\n", t_nt, t_c);
        h->orow.cached = h->ocol.cached = t_c < 0.99 * t_nt;
    }
    for (int d = 0; d < 2; ++d) {
        OrientRT &o = d == 0 ? h->orow : h->ocol;
        double best = 1e30;
        int best_B = 0, best_ept = 8;
        std::vector<int> Bs = {0};
        if ((int64_t)o.gather * h->vbytes > (2 << 20) && o.rows > 0) {
            Bs.push_back(2);
            Bs.push_back(4);
            Bs.push_back(8);
        }
        for (int B : Bs) {
            for (int ept : epts) {
                const double tp = now_s();
                set_plan(h, o, B, ept);
                const double tt = now_s();
                const double ms = timer.time(o, 10);
                if (trace)
                    fprintf(stderr, "tune %s B=%d ept=%d plan %.1f ms run %.3f ms (timing %.1f ms)\n",
                            o.row ? "row" : "col", B, ept, (tt - tp) * 1e3, ms, (now_s() - tt) * 1e3);
                if (ms < best) {
                    best = ms;
                    best_B = B;
                    best_ept = ept;
                }
            }
        }
        // LDS-staged candidates when some instance's gathered vector fits,
        // whole or in up to four slices
        const std::vector<int32_t> &g = o.row ? h->col_off : h->row_off;
        bool any = false, any_slice = false;
        const int64_t vmax = (h->lds_max - SPASS_STATIC_LDS) / h->vbytes - spass_chunk(0);
        for (int32_t q = 0; q < h->count; ++q) {
            any |= g[q + 1] - g[q] <= vmax;
            any_slice |= g[q + 1] - g[q] > vmax / 2 && g[q + 1] - g[q] <= 4 * vmax;
        }
        int best_nnz = 0, best_var = 0, best_slice = 0, best_half = 0;
        if ((any || any_slice) && o.rows > 0) {
            for (int half = 0; half < 2; ++half)
                for (int slice = 0; slice < (any_slice || half ? 2 : 1); ++slice)
                    for (int var = 0; var < 4; ++var)
                        for (int nnz : {16384, 32768, 65536, 131072}) {
                            const double tp = now_s();
                            set_staged(h, o, best_ept, nnz, var, slice, half);
                            const double tt = now_s();
                            if (!o.staged || (slice && !o.sliced)) continue;
                            const double ms = timer.time(o, 10);
                            if (trace)
                                fprintf(stderr, "tune %s staged half=%d slice=%d var=%d nnz=%d plan %.1f ms run "
                                        "%.3f ms (timing %.1f ms)\n", o.row ? "row" : "col", half, slice, var, nnz,
                                        (tt - tp) * 1e3, ms, (now_s() - tt) * 1e3);
                            if (ms < best) {
                                best = ms;
                                best_nnz = nnz;
                                best_var = var;
                                best_slice = slice;
                                best_half = half;
                                best_B = -1;
                            }
                        }
        }
        // direct staged candidates when some instance's whole gathered
        // vector fits in the LDS with nothing beside it; they must beat the
        // others by 3 % of the paired time (on the pump batch direct row
        // passes timed up to 5 % faster alone made the whole iteration 2-4 %
        // slower; paired, the two layouts time within 1 %)
        const int64_t dmax = (h->lds_max - 1024) / h->vbytes;
        const std::vector<int32_t> &off = o.row ? h->row_off : h->col_off;
        bool any_direct = false;
        for (int32_t q = 0; q < h->count; ++q) any_direct |= g[q + 1] - g[q] <= dmax && off[q + 1] > off[q];
        int best_dnnz = 0, best_dl = 1;
        if (any_direct && o.rows > 0) {
            for (int lanes : {2, 4, 8, 16})
                for (int nnz : {32768, 65536}) {
                    const double tp = now_s();
                    set_direct(h, o, best_ept, nnz, lanes);
                    const double tt = now_s();
                    if (!o.direct) continue;
                    const double ms = timer.time(o, 10);
                    if (trace)
                        fprintf(stderr, "tune %s direct lanes=%d nnz=%d plan %.1f ms run %.3f ms (timing %.1f ms)\n",
                                o.row ? "row" : "col", lanes, nnz, (tt - tp) * 1e3, ms, (now_s() - tt) * 1e3);
                    if (ms < 0.97 * best) {
                        best = ms / 0.97;
                        best_dnnz = nnz;
                        best_dl = lanes;
                        best_B = -2;
                    }
                }
        }
        if (best_B == -2) {
            set_direct(h, o, best_ept, best_dnnz, best_dl);
            drop_blocked(o);
            release_sliced(o);
        } else if (best_B < 0) {
            set_staged(h, o, best_ept, best_nnz, best_var, best_slice, best_half);
            drop_blocked(o);
        } else {
            set_plan(h, o, best_B, best_ept);
            if (best_B == 0) drop_blocked(o);
            release_sliced(o);
        }
    }
    // Matrix load policy of the iteration passes: non-temporal, or plain
    // loads that the device's last-level cache keeps across iterations when
    // an iteration's data fits (a gain there, a loss when the data
    // overflows it and evicts itself).  Both passes are timed together,
    // since what the cache keeps depends on both orientations' data.
    if (h->vbytes == 4) {
        double best = 1e30;
        int best_c = 0;
        for (int c : {0, 3, 1, 2}) {  // bit 0: row pass, bit 1: column pass
            h->orow.cached = (c & 1) != 0;
            h->ocol.cached = (c & 2) != 0;
            const double ms = timer.time(h->orow, 20);
            if (trace) fprintf(stderr, "tune cached loads row=%d col=%d run %.3f ms\n", c & 1, (c >> 1) & 1, ms);
            // plain loads must win by 1 %
            if (ms < (c == 0 ? best : 0.99 * best)) {
                best = c == 0 ? ms : ms / 0.99;
                best_c = c;
            }
        }
        h->orow.cached = (best_c & 1) != 0;
        h->ocol.cached = (best_c & 2) != 0;
    }
    refresh_info(h);
    invalidate_graph(h);
    h->tuned = true;
    tune_store(key, current_choice(h));
}

template <class V>
void setup_device(scylla_batch *h, const scylla_lp *lps, HostOrient &csr, HostOrient &csc)
{
    hipStream_t s = h->stream;
    const int32_t M = h->M, N = h->N;
    // matrix: both orientations in their normal layout
    for (int d = 0; d < 2; ++d) {
        OrientRT &o = d == 0 ? h->orow : h->ocol;
        o.row = d == 0;
        o.host = std::move(d == 0 ? csr : csc);
        o.rows = o.host.rows;
        o.gather = d == 0 ? N : M;
        upload(o.ptr, o.host.ptr, s);
        upload(o.ent, o.host.ent, s);
        upload_vals(h, o.val, o.host.v16, o.host.v32, o.host.v64);
        o.mat = MatView{o.ptr.as<int32_t>(), o.ent.as<uint32_t>(), o.val.p, o.host.shift, o.host.mask};
    }
    // FP64 problem vectors (concatenated)
    std::vector<double> c(N), l(N), u(N), b(M);
    std::vector<uint8_t> sn(M);
    for (int32_t q = 0; q < h->count; ++q) {
        const scylla_lp &lp = lps[q];
        memcpy(c.data() + h->col_off[q], lp.c, sizeof(double) * lp.A.n);
        memcpy(l.data() + h->col_off[q], lp.l, sizeof(double) * lp.A.n);
        memcpy(u.data() + h->col_off[q], lp.u, sizeof(double) * lp.A.n);
        if (lp.A.m > 0) {
            memcpy(b.data() + h->row_off[q], lp.b, sizeof(double) * lp.A.m);
            memcpy(sn.data() + h->row_off[q], lp.senses, lp.A.m);
        }
    }
    h->hb = b;
    h->hl = l;
    h->hu = u;
    h->hc = c;
    h->hsense.assign(sn.begin(), sn.end());
    upload(h->c64, c, s);
    upload(h->corig64, c, s);
    upload(h->l64, l, s);
    upload(h->u64, u, s);
    upload(h->b64, b, s);
    upload(h->sense, sn, s);
    const size_t vb = sizeof(V);
    for (DevMem *d : {&h->x, &h->xbar, &h->xr, &h->cv, &h->lv, &h->uv, &h->dc2}) d->alloc((size_t)N * vb);
    for (DevMem *d : {&h->y, &h->yr, &h->b_v, &h->dr2, &h->yp}) d->alloc((size_t)M * vb);
    h->ax.alloc((size_t)M * 8);  // running A x of the adaptive steps, FP64
    h->xp.alloc((size_t)std::max(N, 1) * vb);
    h->axp.alloc((size_t)std::max(M, 1) * 8);
    h->atyp.alloc((size_t)std::max(N, 1) * 8);
    for (DevMem *d : {&h->xp, &h->yp, &h->axp, &h->atyp}) HIPC(hipMemsetAsync(d->p, 0, d->bytes, s));
    for (DevMem *d : {&h->x, &h->xbar, &h->xr}) HIPC(hipMemsetAsync(d->p, 0, d->bytes, s));
    for (DevMem *d : {&h->y, &h->yr, &h->ax}) HIPC(hipMemsetAsync(d->p, 0, d->bytes, s));
    launch_cast<V>(h->c64.as<double>(), h->cv.as<V>(), N, s);
    launch_cast<V>(h->l64.as<double>(), h->lv.as<V>(), N, s);
    launch_cast<V>(h->u64.as<double>(), h->uv.as<V>(), N, s);
    launch_cast<V>(h->b64.as<double>(), h->b_v.as<V>(), M, s);
    // bounds shared by every column of an instance (binary problems): the
    // column pass then reads them once per workgroup, not per column
    {
        std::vector<V> ib(2 * (size_t)h->count, std::numeric_limits<V>::quiet_NaN());
        for (int32_t q = 0; q < h->count; ++q) {
            const int32_t j0 = h->col_off[q], j1 = h->col_off[q + 1];
            bool uni = j1 > j0;
            for (int32_t j = j0 + 1; j < j1 && uni; ++j) uni = l[j] == l[j0] && u[j] == u[j0];
            if (uni) {
                ib[2 * q] = (V)l[j0];
                ib[2 * q + 1] = (V)u[j0];
            }
        }
        upload(h->ibnd, ib, s);
    }
    // preconditioner: 10 Ruiz rounds (infinity norm) + one Pock-Chambolle
    // round (alpha = 1), FP64; A itself stays unscaled
    std::vector<double> ones_m(M, 1.0), ones_n(N, 1.0);
    upload(h->dr64, ones_m, s);
    upload(h->dc64, ones_n, s);
    DevMem rt, ct;
    rt.alloc((size_t)std::max(M, 1) * 8);
    ct.alloc((size_t)std::max(N, 1) * 8);
    for (int it = 0; it < 11; ++it) {
        const int mode = it < 10 ? 0 : 1;
        launch_scale_reduce(h->orow.mat, h->fmt, M, h->dr64.as<double>(), h->dc64.as<double>(), rt.as<double>(), mode, s);
        launch_scale_reduce(h->ocol.mat, h->fmt, N, h->dc64.as<double>(), h->dr64.as<double>(), ct.as<double>(), mode, s);
        launch_scale_apply(h->dr64.as<double>(), rt.as<double>(), M, s);
        launch_scale_apply(h->dc64.as<double>(), ct.as<double>(), N, s);
    }
    launch_finish_diag<V>(h->dr64.as<double>(), h->dr2.as<V>(), M, s);
    launch_finish_diag<V>(h->dc64.as<double>(), h->dc2.as<V>(), N, s);
    // states and norms
    std::vector<InstState> st(h->count);
    memset(st.data(), 0, sizeof(InstState) * st.size());
    for (auto &S : st) S.status = ST_ITER;  // idle until the first solve
    upload(h->st, st, s);
    set_plan(h, h->orow, 0, 8);
    set_plan(h, h->ocol, 0, 8);
    refresh_info(h);
    launch_inst_norms(h->info.as<InstInfo>(), h->count, h->b64.as<double>(), h->c64.as<double>(),
                      h->dr64.as<double>(), h->dc64.as<double>(), h->st.as<InstState>(), s);
    HIPC(hipGetLastError());
    // fused-window eligibility: every instance fits in LDS
    size_t need = 0;
    for (int32_t q = 0; q < h->count; ++q) {
        const int32_t m = h->row_off[q + 1] - h->row_off[q], n = h->col_off[q + 1] - h->col_off[q];
        const int32_t rn = h->orow.host.ptr[h->row_off[q + 1]] - h->orow.host.ptr[h->row_off[q]];
        const int32_t cn = h->ocol.host.ptr[h->col_off[q + 1]] - h->ocol.host.ptr[h->col_off[q]];
        need = std::max(need, tiny_lds_bytes(m, n, rn, cn, (int)sizeof(V)));
    }
    h->tiny_ok = need + 1024 <= (size_t)h->lds_max;  // room for the kernel's static LDS
    h->tiny_shmem = need;
    if (h->tiny_ok) {
        TinyArgs<V> a{};
        launch_tiny<V>(a, h->fmt, h->count, 1, need, s, true);
    }
    HIPC(hipStreamSynchronize(s));
}

}  // namespace

namespace scy {

int fail_code(const Err &e)
{
    g_err = e.msg;
    return e.code;
}

int validate_params(const scylla_params *p)
{
    if (!p) throw_err(-EINVAL, "params is NULL");
    if (!(p->tol > 0.0) && !(p->tol <= 0.0)) throw_err(-EINVAL, "tol is NaN");
    if (p->iter_limit < 0) throw_err(-EINVAL, "iter_limit < 0");
    if (p->check_period < 1 || p->check_period > 1024) throw_err(-EINVAL, "check_period must be in [1, 1024]");
    if (!(p->eta > 0.0 && p->eta < 1.0)) throw_err(-EINVAL, "eta must be in (0, 1)");
    if (p->precision != SCYLLA_FP32 && p->precision != SCYLLA_FP64) throw_err(-EINVAL, "bad precision");
    if (p->adaptive != 0 && p->adaptive != 1) throw_err(-EINVAL, "adaptive must be 0 or 1");
    if (p->restart_avg != 0 && p->restart_avg != 1) throw_err(-EINVAL, "restart_avg must be 0 or 1");
    if (p->compact != 0 && p->compact != 1) throw_err(-EINVAL, "compact must be 0 or 1");
    if (!(p->infeas_tol >= 0.0) || !isfinite(p->infeas_tol)) throw_err(-EINVAL, "infeas_tol must be finite and >= 0");
    if (!(p->stall_tol >= 0.0) || !isfinite(p->stall_tol)) throw_err(-EINVAL, "stall_tol must be finite and >= 0");
    if (p->stall_tol > 0.0 && p->stall_checks < 1) throw_err(-EINVAL, "stall_checks must be >= 1");
    return 0;
}

void check_inst(scylla_batch *h, int32_t inst)
{
    if (!h) throw_err(-EINVAL, "handle is NULL");
    if (inst < 0 || inst >= h->count) throw_err(-EINVAL, "instance index out of range");
}

template <class V>
void project_start(scylla_batch *h, int32_t inst, int zero)
{
    const int clo = inst < 0 ? 0 : h->col_off[inst], chi = inst < 0 ? h->N : h->col_off[inst + 1];
    const int rlo = inst < 0 ? 0 : h->row_off[inst], rhi = inst < 0 ? h->M : h->row_off[inst + 1];
    launch_project<V>(h->x.as<V>(), h->lv.as<V>(), h->uv.as<V>(), clo, chi, h->y.as<V>(),
                      h->sense.as<uint8_t>(), rlo, rhi, zero, h->stream);
}

// Projects (after zeroing, when `zero`) the start points of instances
// [q0, q1), which occupy contiguous column and row ranges.
template <class V>
void project_range(scylla_batch *h, int32_t q0, int32_t q1, int zero)
{
    launch_project<V>(h->x.as<V>(), h->lv.as<V>(), h->uv.as<V>(), h->col_off[q0], h->col_off[q1], h->y.as<V>(),
                      h->sense.as<uint8_t>(), h->row_off[q0], h->row_off[q1], zero, h->stream);
}

void read_states(scylla_batch *h, std::vector<InstState> &out)
{
    out.resize(h->count);
    HIPC(hipMemcpyAsync(out.data(), h->st.p, sizeof(InstState) * h->count, hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
}

void fill_result(const InstState &S, scylla_result &r, double solve_s, double setup_s)
{
    memset(&r, 0, sizeof(r));
    r.status = S.status;
    r.restarts = S.restarts;
    r.iterations = S.k;
    r.rel_kkt = S.rel;
    r.rho_primal = S.rho_p;
    r.rho_dual = S.rho_d;
    r.rho_gap = S.rho_g;
    r.primal_obj = S.pobj;
    r.dual_obj = S.dobj;
    r.omega = S.omega;
    r.solve_seconds = solve_s;
    r.setup_seconds = setup_s;
}

int batch_solve_impl(scylla_batch *h, const scylla_params *p, int32_t warm, scylla_result *results,
                     const int64_t *k_limits, int32_t q0, int32_t q1)
{
    if (q1 < 0) q1 = h ? h->count : 0;
    if (!h || !results) throw_err(-EINVAL, "handle or results is NULL");
    validate_params(p);
    if (p->precision != h->precision) throw_err(-EINVAL, "params precision differs from the handle's");
    // the fused window has no running average: restart to the average takes
    // the per-pass path
    const bool tiny = h->tiny_ok && p->fused_window != 0 && p->restart_avg == 0;
    h->adaptive = p->adaptive != 0;
    h->avg_on = p->restart_avg != 0;
    if (h->avg_on) {
        const size_t vb = (size_t)h->vbytes;
        if (h->xavg.bytes < (size_t)std::max(h->N, 1) * vb) h->xavg.alloc((size_t)std::max(h->N, 1) * vb);
        if (h->yavg.bytes < (size_t)std::max(h->M, 1) * vb) h->yavg.alloc((size_t)std::max(h->M, 1) * vb);
        if (h->adaptive && h->axavg.bytes < (size_t)std::max(h->M, 1) * 8)
            h->axavg.alloc((size_t)std::max(h->M, 1) * 8);
    }
    double tune_s = 0.0;
    if (p->autotune && !h->tuned && !tiny) {
        const double tt = now_s();
        if (h->vbytes == 4) autotune<float>(h);
        else autotune<double>(h);
        tune_s = now_s() - tt;
    }
    std::vector<InstState> st;
    read_states(h, st);
    for (int32_t q = 0; q < h->count; ++q) {
        InstState &S = st[q];
        if (k_limits && k_limits[q] <= 0) {
            if (S.status == ST_RUN) S.status = ST_ITER;
            continue;
        }
        const double omega = (warm && S.omega > 0.0) ? S.omega : S.omega0;
        S.status = ST_RUN;
        S.nrun = 0;
        S.restarts = 0;
        S.restart_now = 0;
        S.restart_on = p->restarts ? 1 : 0;
        S.avg_on = p->restart_avg ? 1 : 0;
        S.take_avg = 0;
        S.force_stop = 0;
        S.k = 0;
        S.k_limit = k_limits ? std::min<int64_t>(k_limits[q], p->iter_limit) : p->iter_limit;
        S.kr = 0;
        S.omega = omega;
        S.eta = p->eta;
        S.t = p->eta / omega;
        S.s = p->eta * omega;
        S.tol = p->tol;
        S.infeas_tol = p->infeas_tol;
        S.stall_tol = p->stall_tol;
        S.stall_checks = p->stall_checks;
        S.nstall = 0;
        S.pprev = S.dprev = 0.0;
        S.Er = S.Ep = 0.0;
        S.rel = S.rho_p = S.rho_d = S.rho_g = S.pobj = S.dobj = 0.0;
    }
    if (q1 > q0) {
        if (h->vbytes == 4) project_range<float>(h, q0, q1, warm ? 0 : 1);
        else project_range<double>(h, q0, q1, warm ? 0 : 1);
    }
    HIPC(hipMemcpyAsync(h->st.p, st.data(), sizeof(InstState) * h->count, hipMemcpyHostToDevice, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    ensure_graph(h, p->check_period, tiny);

    // cutting finished instances out of the iteration launches (results
    // unchanged); the full lists come back when the solve ends
    struct Restore {
        scylla_batch *h;
        ~Restore() { uncut(h); }
    } restore{h};
    const bool can_cut = p->compact != 0 && !tiny && (iter_tiles(h->orow, nullptr) + iter_tiles(h->ocol, nullptr)) > 0;
    const bool cut_trace = getenv("SCYLLA_CUT_TRACE") != nullptr;
    std::vector<uint8_t> run(h->count, 0);
    int64_t graph_tiles = 0, cut_after = -1, next = 0;
    auto maybe_cut = [&](int64_t window) {
        const int64_t live = iter_tiles(h->orow, run.data()) + iter_tiles(h->ocol, run.data());
        // at most half the launched tiles still run, and at least 16 fewer
        if (live * 2 > graph_tiles || graph_tiles - live < 16) return;
        cut_after = next;  // the first window launched over the cut lists
        const double tc = now_s();
        cut_lists(h, run.data());
        if (h->cexec) h->retired.push_back(h->cexec);
        h->cexec = nullptr;
        h->cexec = capture_window(h, p->check_period, false);
        if (cut_trace)
            fprintf(stderr, "cut after window %lld: %lld -> %lld tiles, %.2f ms on the host\n", (long long)window,
                    (long long)graph_tiles, (long long)live, (now_s() - tc) * 1e3);
        graph_tiles = live;
    };
    if (can_cut) {
        prepare_cut(h);
        graph_tiles = iter_tiles(h->orow, nullptr) + iter_tiles(h->ocol, nullptr);
        for (int32_t q = 0; q < h->count; ++q) run[q] = st[q].status == ST_RUN ? 1 : 0;
        maybe_cut(-1);  // instances with no iterations in this solve
    }

    const size_t sb = sizeof(InstState) * (size_t)h->count;
    const double t0 = now_s();
    int64_t insp = 0;
    bool done = false, forced = false;
    int64_t last_slot = 0;
    for (;;) {
        while (!done && next - insp < 2) {
            const int slot = (int)(next & 1);
            HIPC(hipGraphLaunch(h->cexec ? h->cexec : h->gexec, h->stream));
            HIPC(hipMemcpyAsync(h->pinned + (size_t)slot * h->count, h->st.p, sb, hipMemcpyDeviceToHost, h->stream));
            HIPC(hipEventRecord(h->ev[slot], h->stream));
            ++next;
        }
        if (insp == next) break;
        const int slot = (int)(insp & 1);
        HIPC(hipEventSynchronize(h->ev[slot]));
        last_slot = slot;
        ++insp;
        bool running = false;
        for (int32_t q = 0; q < h->count; ++q)
            if (h->pinned[(size_t)slot * h->count + q].status == ST_RUN) running = true;
        if (!running) {
            done = true;
        } else if (!forced && p->time_limit_s > 0.0 && now_s() - t0 > p->time_limit_s) {
            launch_force_stop(h->st.as<InstState>(), h->count, h->stream);
            HIPC(hipGetLastError());
            forced = true;
        } else if (can_cut && insp > cut_after) {
            // the staging of the last cut is free once a window launched
            // behind its copies has been inspected
            for (int32_t q = 0; q < h->count; ++q)
                run[q] = h->pinned[(size_t)slot * h->count + q].status == ST_RUN ? 1 : 0;
            maybe_cut(insp - 1);
        }
    }
    HIPC(hipStreamSynchronize(h->stream));
    const double solve_s = now_s() - t0;
    for (int32_t q = 0; q < h->count; ++q) {
        fill_result(h->pinned[(size_t)last_slot * h->count + q], results[q], solve_s, h->setup_seconds);
        results[q].tune_seconds = tune_s;
    }
    return 0;
}

// Allocates the diagonal Hessian (zero) on first use; the kernels then take
// the QP form of the primal step, so the graph is rebuilt.
void ensure_q(scylla_batch *h)
{
    if (h->has_q) return;
    h->q64.alloc((size_t)std::max(h->N, 1) * 8);
    h->qv.alloc((size_t)std::max(h->N, 1) * h->vbytes);
    HIPC(hipMemsetAsync(h->q64.p, 0, h->q64.bytes, h->stream));
    HIPC(hipMemsetAsync(h->qv.p, 0, h->qv.bytes, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    h->has_q = true;
    invalidate_graph(h);
}

void cast_q(scylla_batch *h)
{
    if (h->vbytes == 4) launch_cast<float>(h->q64.as<double>(), h->qv.as<float>(), h->N, h->stream);
    else launch_cast<double>(h->q64.as<double>(), h->qv.as<double>(), h->N, h->stream);
}

}  // namespace scy

// =================================================================== C ABI
extern "C" {

int scylla_params_default(scylla_params *p)
{
    if (!p) {
        g_err = "params is NULL";
        return -EINVAL;
    }
    p->tol = 1e-4;
    p->iter_limit = 100000;
    p->precision = SCYLLA_FP32;
    p->check_period = 64;
    p->restarts = 1;
    p->autotune = 1;
    p->eta = 0.99;
    p->time_limit_s = 0.0;
    p->fused_window = 1;
    p->adaptive = 0;
    p->infeas_tol = 1e-8;
    p->stall_tol = 0.0;
    p->stall_checks = 3;
    p->restart_avg = 0;
    p->compact = 1;
    return 0;
}

const char *scylla_last_error(void) { return g_err.c_str(); }

int scylla_validate_lp(const scylla_lp *lp)
{
    return guarded([&]() {
        std::string err;
        int rc = validate_lp(lp, err);
        if (rc) throw_err(rc, err);
        return 0;
    });
}

int scylla_batch_create(const scylla_lp *lps, int32_t count, int32_t precision, void *hip_stream,
                        scylla_batch **out)
{
    return guarded([&]() {
        if (!out) throw_err(-EINVAL, "out is NULL");
        *out = nullptr;
        if (!lps || count < 1) throw_err(-EINVAL, "need at least one LP");
        if (precision != SCYLLA_FP32 && precision != SCYLLA_FP64) throw_err(-EINVAL, "bad precision");
        std::string err;
        for (int32_t q = 0; q < count; ++q) {
            int rc = validate_lp(&lps[q], err);
            if (rc) throw_err(rc, "instance " + std::to_string(q) + ": " + err);
        }
        const double t0 = now_s();
        auto h = std::make_unique<scylla_batch>();
        h->count = count;
        h->precision = precision;
        h->vbytes = precision == SCYLLA_FP32 ? 4 : 8;
        HostOrient csr, csc;
        int32_t fmt = 0;
        int rc = build_orientations(lps, count, precision, csr, csc, fmt, h->row_off, h->col_off, err);
        if (rc) throw_err(rc, err);
        h->fmt = fmt;
        h->M = csr.rows;
        h->N = csc.rows;
        h->NNZ = (int64_t)csr.ent.size();
        check_device();
        {
            int dev = 0, lds = 0;
            HIPC(hipGetDevice(&dev));
            HIPC(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            h->lds_max = lds;
        }
        if (hip_stream) {
            h->stream = (hipStream_t)hip_stream;
        } else {
            HIPC(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            h->own_stream = true;
        }
        HIPC(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIPC(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        HIPC(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
        HIPC(hipEventCreateWithFlags(&h->join, hipEventDisableTiming));
        HIPC(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
        HIPC(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
        HIPC(hipHostMalloc((void **)&h->pinned, sizeof(InstState) * 2 * (size_t)count, hipHostMallocDefault));
        if (h->vbytes == 4) setup_device<float>(h.get(), lps, csr, csc);
        else setup_device<double>(h.get(), lps, csr, csc);
        h->hval.resize(h->NNZ);
        for (int32_t q = 0, e = 0; q < count; ++q) {
            memcpy(h->hval.data() + e, lps[q].A.val, sizeof(double) * lps[q].A.nnz);
            e += (int32_t)lps[q].A.nnz;
        }
        h->setup_seconds = now_s() - t0;
        *out = h.release();
        return 0;
    });
}

void scylla_batch_destroy(scylla_batch *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    delete h;
}

int scylla_batch_set_objective(scylla_batch *h, int32_t inst, const double *c_hat)
{
    return guarded([&]() {
        check_inst(h, inst);
        if (!c_hat) throw_err(-EINVAL, "c_hat is NULL");
        const int32_t lo = h->col_off[inst], len = h->col_off[inst + 1] - lo;
        for (int32_t j = 0; j < len; ++j)
            if (!isfinite(c_hat[j])) throw_err(-EINVAL, "non-finite objective");
        HIPC(hipMemcpyAsync(h->c64.as<double>() + lo, c_hat, sizeof(double) * len, hipMemcpyHostToDevice, h->stream));
        if (h->vbytes == 4) launch_cast<float>(h->c64.as<double>(), h->cv.as<float>(), h->N, h->stream);
        else launch_cast<double>(h->c64.as<double>(), h->cv.as<double>(), h->N, h->stream);
        launch_inst_norms(h->info.as<InstInfo>(), h->count, h->b64.as<double>(), h->c64.as<double>(),
                          h->dr64.as<double>(), h->dc64.as<double>(), h->st.as<InstState>(), h->stream);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_batch_set_quadratic(scylla_batch *h, int32_t inst, const double *q)
{
    return guarded([&]() {
        check_inst(h, inst);
        const int32_t lo = h->col_off[inst], len = h->col_off[inst + 1] - lo;
        if (q)
            for (int32_t j = 0; j < len; ++j)
                if (!(q[j] >= 0.0) || !isfinite(q[j])) throw_err(-EINVAL, "q must be finite and >= 0");
        if (!q && !h->has_q) return 0;
        ensure_q(h);
        if (q) {
            HIPC(hipMemcpyAsync(h->q64.as<double>() + lo, q, sizeof(double) * len, hipMemcpyHostToDevice,
                                h->stream));
        } else {
            HIPC(hipMemsetAsync(h->q64.as<double>() + lo, 0, sizeof(double) * len, h->stream));
        }
        cast_q(h);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_batch_set_blend(scylla_batch *h, int32_t inst, const uint8_t *xhat_bits, const uint8_t *int_bits,
                           double a, double kappa)
{
    return guarded([&]() {
        check_inst(h, inst);
        if (!xhat_bits) throw_err(-EINVAL, "xhat_bits is NULL");
        if (!isfinite(a) || !isfinite(kappa)) throw_err(-EINVAL, "a and kappa must be finite");
        const int32_t lo = h->col_off[inst], hi = h->col_off[inst + 1];
        const size_t nb = (size_t)(hi - lo + 7) / 8;
        if (h->bits_tmp.bytes < nb) h->bits_tmp.alloc(nb);
        if (int_bits && h->ibits_tmp.bytes < nb) h->ibits_tmp.alloc(nb);
        HIPC(hipMemcpyAsync(h->bits_tmp.p, xhat_bits, nb, hipMemcpyHostToDevice, h->stream));
        if (int_bits) HIPC(hipMemcpyAsync(h->ibits_tmp.p, int_bits, nb, hipMemcpyHostToDevice, h->stream));
        const uint8_t *ib = int_bits ? h->ibits_tmp.as<uint8_t>() : nullptr;
        if (h->vbytes == 4)
            launch_blend<float>(h->corig64.as<double>(), h->bits_tmp.as<uint8_t>(), ib, a, kappa,
                                h->c64.as<double>(), h->cv.as<float>(), lo, hi, h->stream);
        else
            launch_blend<double>(h->corig64.as<double>(), h->bits_tmp.as<uint8_t>(), ib, a, kappa,
                                 h->c64.as<double>(), h->cv.as<double>(), lo, hi, h->stream);
        launch_inst_norms(h->info.as<InstInfo>(), h->count, h->b64.as<double>(), h->c64.as<double>(),
                          h->dr64.as<double>(), h->dc64.as<double>(), h->st.as<InstState>(), h->stream);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_batch_set_start(scylla_batch *h, int32_t inst, const double *x0, const double *y0, double omega0)
{
    return guarded([&]() {
        check_inst(h, inst);
        const int32_t clo = h->col_off[inst], clen = h->col_off[inst + 1] - clo;
        const int32_t rlo = h->row_off[inst], rlen = h->row_off[inst + 1] - rlo;
        if (x0)
            for (int32_t j = 0; j < clen; ++j)
                if (isnan(x0[j])) throw_err(-EINVAL, "NaN in x0");
        if (y0)
            for (int32_t i = 0; i < rlen; ++i)
                if (!isfinite(y0[i])) throw_err(-EINVAL, "non-finite y0");
        if (h->vbytes == 4) {
            if (x0) put_range<float>(h, h->x, clo, clen, x0);
            if (y0) put_range<float>(h, h->y, rlo, rlen, y0);
            project_start<float>(h, inst, 0);
        } else {
            if (x0) put_range<double>(h, h->x, clo, clen, x0);
            if (y0) put_range<double>(h, h->y, rlo, rlen, y0);
            project_start<double>(h, inst, 0);
        }
        if (omega0 > 0.0) {
            std::vector<InstState> st;
            read_states(h, st);
            st[inst].omega = omega0;
            HIPC(hipMemcpyAsync(h->st.as<InstState>() + inst, &st[inst], sizeof(InstState), hipMemcpyHostToDevice,
                                h->stream));
        }
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_batch_set_start_device(scylla_batch *h, const double *x0_dev, const double *y0_dev,
                                  const double *omega0)
{
    return guarded([&]() {
        if (!h) throw_err(-EINVAL, "handle is NULL");
        if (omega0)
            for (int32_t q = 0; q < h->count; ++q)
                if (!(omega0[q] <= 0.0 || isfinite(omega0[q]))) throw_err(-EINVAL, "non-finite omega0");
        // validated on the device before anything is written
        if (x0_dev || y0_dev) {
            if (h->start_flag.bytes < sizeof(int)) h->start_flag.alloc(sizeof(int));
            HIPC(hipMemsetAsync(h->start_flag.p, 0, sizeof(int), h->stream));
            launch_start_check(x0_dev, h->N, y0_dev, h->M, h->start_flag.as<int>(), h->stream);
            HIPC(hipGetLastError());
            int bad = 0;
            HIPC(hipMemcpyAsync(&bad, h->start_flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIPC(hipStreamSynchronize(h->stream));
            if (bad & 1) throw_err(-EINVAL, "NaN in x0");
            if (bad & 2) throw_err(-EINVAL, "non-finite y0");
        }
        if (h->vbytes == 4) {
            if (x0_dev) launch_cast<float>(x0_dev, h->x.as<float>(), h->N, h->stream);
            if (y0_dev) launch_cast<float>(y0_dev, h->y.as<float>(), h->M, h->stream);
            project_range<float>(h, 0, h->count, 0);
        } else {
            if (x0_dev) launch_cast<double>(x0_dev, h->x.as<double>(), h->N, h->stream);
            if (y0_dev) launch_cast<double>(y0_dev, h->y.as<double>(), h->M, h->stream);
            project_range<double>(h, 0, h->count, 0);
        }
        if (omega0) {
            std::vector<InstState> st;
            read_states(h, st);
            for (int32_t q = 0; q < h->count; ++q)
                if (omega0[q] > 0.0) st[q].omega = omega0[q];
            HIPC(hipMemcpyAsync(h->st.p, st.data(), sizeof(InstState) * h->count, hipMemcpyHostToDevice,
                                h->stream));
        }
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_batch_solve(scylla_batch *h, const scylla_params *p, int32_t warm, scylla_result *results)
{
    return guarded([&]() { return batch_solve_impl(h, p, warm, results); });
}

int scylla_batch_get_solution(scylla_batch *h, int32_t inst, double *x, double *y)
{
    return guarded([&]() {
        check_inst(h, inst);
        const int32_t clo = h->col_off[inst], clen = h->col_off[inst + 1] - clo;
        const int32_t rlo = h->row_off[inst], rlen = h->row_off[inst + 1] - rlo;
        if (h->vbytes == 4) {
            get_range<float>(h, h->x, clo, clen, x);
            get_range<float>(h, h->y, rlo, rlen, y);
        } else {
            get_range<double>(h, h->x, clo, clen, x);
            get_range<double>(h, h->y, rlo, rlen, y);
        }
        return 0;
    });
}

int scylla_batch_get_average(scylla_batch *h, int32_t inst, double *x, double *y)
{
    return guarded([&]() {
        check_inst(h, inst);
        if (!h->xavg.p || !h->yavg.p) throw_err(-EINVAL, "no solve with restart_avg has run on this handle");
        const int32_t clo = h->col_off[inst], clen = h->col_off[inst + 1] - clo;
        const int32_t rlo = h->row_off[inst], rlen = h->row_off[inst + 1] - rlo;
        if (h->vbytes == 4) {
            get_range<float>(h, h->xavg, clo, clen, x);
            get_range<float>(h, h->yavg, rlo, rlen, y);
        } else {
            get_range<double>(h, h->xavg, clo, clen, x);
            get_range<double>(h, h->yavg, rlo, rlen, y);
        }
        return 0;
    });
}

int scylla_batch_get_x_all(scylla_batch *h, double *x_all)
{
    return guarded([&]() {
        if (!h || !x_all) throw_err(-EINVAL, "handle or x_all is NULL");
        if (h->vbytes == 4) get_range<float>(h, h->x, 0, h->N, x_all);
        else get_range<double>(h, h->x, 0, h->N, x_all);
        return 0;
    });
}

int scylla_batch_device_iterates(scylla_batch *h, void **x, void **y, int32_t *elem_bytes)
{
    return guarded([&]() {
        if (!h || !x || !y || !elem_bytes) throw_err(-EINVAL, "NULL argument");
        *x = h->x.p;
        *y = h->y.p;
        *elem_bytes = h->vbytes;
        return 0;
    });
}

int scylla_batch_get_info(scylla_batch *h, scylla_batch_info *info)
{
    return guarded([&]() {
        if (!h || !info) throw_err(-EINVAL, "NULL argument");
        memset(info, 0, sizeof(*info));
        info->count = h->count;
        info->precision = h->precision;
        info->format = h->fmt;
        info->fused_eligible = h->tiny_ok ? 1 : 0;
        info->m_total = h->M;
        info->n_total = h->N;
        info->nnz_total = h->NNZ;
        info->row_chunk = 256 * std::abs(h->orow.ept);
        info->col_chunk = 256 * std::abs(h->ocol.ept);
        info->row_tile_threads = h->orow.ept < 0 ? 1024 : 256;
        info->col_tile_threads = h->ocol.ept < 0 ? 1024 : 256;
        info->long_rows = h->orow.nlong();
        info->long_cols = h->ocol.nlong();
        info->row_blocks = h->orow.direct ? -6 : (h->orow.staged ? -1 : (h->orow.blocked ? h->orow.bh.B : 0));
        info->col_blocks = h->ocol.direct ? -6 : (h->ocol.staged ? -1 : (h->ocol.blocked ? h->ocol.bh.B : 0));
        info->row_staged_nnz = h->orow.staged ? h->orow.staged_nnz : 0;
        info->col_staged_nnz = h->ocol.staged ? h->ocol.staged_nnz : 0;
        info->row_staged_variant = h->orow.staged ? h->orow.svariant : 0;
        info->col_staged_variant = h->ocol.staged ? h->ocol.svariant : 0;
        for (int32_t q = 0; q < h->count; ++q) {
            info->row_sliced += h->orow.sliced && h->orow.xplan.sliced[q];
            info->col_sliced += h->ocol.sliced && h->ocol.xplan.sliced[q];
        }
        info->row_slices = h->orow.sliced ? h->orow.xplan.S : 0;
        info->col_slices = h->ocol.sliced ? h->ocol.xplan.S : 0;
        info->row_half_lds = h->orow.staged && h->orow.shalf;
        info->col_half_lds = h->ocol.staged && h->ocol.shalf;
        for (int32_t q = 0; q < h->count; ++q) {
            info->row_direct += h->orow.direct && h->orow.dinst[q];
            info->col_direct += h->ocol.direct && h->ocol.dinst[q];
        }
        info->row_staged_nnz = h->orow.direct ? h->orow.dnnz : info->row_staged_nnz;
        info->col_staged_nnz = h->ocol.direct ? h->ocol.dnnz : info->col_staged_nnz;
        info->row_cached = h->orow.cached ? 1 : 0;
        info->col_cached = h->ocol.cached ? 1 : 0;
        return 0;
    });
}

int scylla_batch_set_cached_loads(scylla_batch *h, int32_t row_cached, int32_t col_cached)
{
    return guarded([&]() {
        if (!h) throw_err(-EINVAL, "handle is NULL");
        if ((row_cached != 0 && row_cached != 1) || (col_cached != 0 && col_cached != 1))
            throw_err(-EINVAL, "flags must be 0 or 1");
        HIPC(hipStreamSynchronize(h->stream));
        h->orow.cached = row_cached != 0 && h->vbytes == 4;
        h->ocol.cached = col_cached != 0 && h->vbytes == 4;
        invalidate_graph(h);
        return 0;
    });
}

int scylla_batch_set_layout(scylla_batch *h, int32_t row_blocks, int32_t row_ept, int32_t col_blocks,
                            int32_t col_ept)
{
    return guarded([&]() {
        if (!h) throw_err(-EINVAL, "handle is NULL");
        auto okB = [](int32_t B) {
            return B == 0 || B == 2 || B == 4 || B == 8 || (B >= -8 && B <= -6) || (B >= -3 && B <= -1);
        };
        auto okE = [](int32_t e) { return e == 2 || e == 4 || e == 8 || e == 16 || e == -8 || e == -16; };
        if (!okB(row_blocks) || !okB(col_blocks) || !okE(row_ept) || !okE(col_ept))
            throw_err(-EINVAL, "blocks must be -8, -7, -6, -3, -2, -1, 0, 2, 4 or 8 and ept 2, 4, 8, 16, -8 or -16");
        HIPC(hipStreamSynchronize(h->stream));
        for (int d = 0; d < 2; ++d) {
            OrientRT &o = d == 0 ? h->orow : h->ocol;
            o.cached = false;  // non-temporal matrix loads unless set otherwise
            int32_t B = d == 0 ? row_blocks : col_blocks, ept = d == 0 ? row_ept : col_ept;
            if (o.rows == 0 && B > 0) B = 0;
            if (B <= -6) {
                // at least 1, 4 or 8 lanes per row (8, 4 or 2 nonzeros per lane and round)
                set_direct(h, o, ept, 32768, B == -6 ? 1 : (B == -7 ? 4 : 8));
                drop_blocked(o);
                release_sliced(o);
            } else if (B < 0) {
                set_staged(h, o, ept, 32768, 0, B <= -2 ? 1 : 0, B == -3 ? 1 : 0);
                drop_blocked(o);
            } else {
                set_plan(h, o, B, ept);
                if (B == 0) drop_blocked(o);
                release_sliced(o);
            }
        }
        refresh_info(h);
        invalidate_graph(h);
        h->tuned = true;
        return 0;
    });
}

int scylla_batch_time_passes(scylla_batch *h, int32_t reps, double *ms_row, double *ms_col)
{
    return guarded([&]() {
        if (!h || !ms_row || !ms_col || reps < 1) throw_err(-EINVAL, "bad argument");
        HIPC(hipStreamSynchronize(h->stream));
        if (h->vbytes == 4) {
            PassTimer<float> t(h);
            *ms_row = t.time(h->orow, reps, false);
            *ms_col = t.time(h->ocol, reps, false);
        } else {
            PassTimer<double> t(h);
            *ms_row = t.time(h->orow, reps, false);
            *ms_col = t.time(h->ocol, reps, false);
        }
        HIPC(hipStreamSynchronize(h->stream));
        return 0;
    });
}

int scylla_pdhg_solve(const scylla_csr *A, const double *c, const double *b, const char *senses, const double *l,
                      const double *u, const scylla_params *p, const double *x0, const double *y0, double *x_out,
                      double *y_out, scylla_result *res)
{
    return guarded([&]() {
        if (!A || !res || !x_out || (A->m > 0 && !y_out)) throw_err(-EINVAL, "NULL argument");
        validate_params(p);
        scylla_lp lp{*A, c, b, senses, l, u};
        std::string err;
        int rc = validate_lp(&lp, err);
        if (rc) throw_err(rc, err);
        scylla_batch *h = nullptr;
        rc = scylla_batch_create(&lp, 1, p->precision, nullptr, &h);
        if (rc) return rc;
        std::unique_ptr<scylla_batch, void (*)(scylla_batch *)> guard(h, scylla_batch_destroy);
        const bool warm = x0 || y0;
        if (warm) {
            rc = scylla_batch_set_start(h, 0, x0, y0, 0.0);
            if (rc) return rc;
        }
        scylla_result r;
        rc = scylla_batch_solve(h, p, warm ? 1 : 0, &r);
        if (rc) return rc;
        rc = scylla_batch_get_solution(h, 0, x_out, y_out);
        if (rc) return rc;
        *res = r;
        return 0;
    });
}

}  // extern "C"
