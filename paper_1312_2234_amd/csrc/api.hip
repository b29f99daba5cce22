// api.hip -- host side of the C ABI declared in include/lbm.h.
//
// Workspace layout (each region 256-byte aligned), all carved from the caller's buffer:
//   channel descriptors | segment -> channel map | populations A | populations B |
//   device error flags | IB: node -> channel, node records, two tile sets (counts,
//   tile -> slot, flagged list, list channel, fill, list offsets, header), node lists,
//   force blocks, velocity blocks.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "lbm_internal.h"

using namespace lbmib;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_params(const lbm_params* p, int32_t nch) {
    if (!p || nch < 1) return false;
    for (int c = 0; c < nch; ++c) {
        const lbm_params& q = p[c];
        if (q.nx < 1 || q.ny < 1 || q.nz < 1) return false;
        if ((int64_t)q.nx * q.ny * q.nz >= (int64_t(1) << 31)) return false;
        if (!(q.tau > 0.5f) || !(q.tau < 1e6f)) return false;
        if (q.walls < 0 || q.walls > 2) return false;
        if (q.walls == 2 && q.ny < 3) return false;  // two wall rows and at least one fluid row
        if (q.u_wall_lo[1] != 0.0f || q.u_wall_hi[1] != 0.0f) return false;
    }
    return true;
}

size_t elem_size(lbm_storage s) { return s == LBM_STORE_F32 ? 4 : 2; }

struct Sizes {
    int64_t cells = 0, segs = 0, tiles = 0, slots = 0, list_cap = 0;
};

Sizes sizes_of(const lbm_params* p, int32_t nch, int64_t max_nodes) {
    Sizes s;
    for (int c = 0; c < nch; ++c) {
        const int64_t n = (int64_t)p[c].nx * p[c].ny * p[c].nz;
        s.cells += n;
        s.segs += (n + 63) / 64;
        s.tiles += (int64_t)((p[c].nx + TILE - 1) / TILE) * ((p[c].ny + TILE - 1) / TILE) * ((p[c].nz + TILE - 1) / TILE);
    }
    if (max_nodes > 0) {
        s.slots = std::min<int64_t>(s.tiles, 27 * max_nodes);
        s.list_cap = 27 * max_nodes;
    }
    return s;
}

// Partial blocks of split spread tiles: a split tile has more than SP_CHUNK nodes, so a list
// of list_cap entries has at most 2 list_cap / SP_CHUNK chunks in split tiles.
int64_t part_cap_of(const Sizes& sz) {
    const int64_t c = 2 * sz.list_cap / SP_CHUNK + 64;
    return c < SP_PART_MAX ? c : SP_PART_MAX;
}

// Spread work items: one per flagged tile plus one per further SP_CHUNK list entries.
int64_t max_items_of(const Sizes& sz) { return sz.slots + sz.list_cap / SP_CHUNK + 1; }

Layout layout_of(const lbm_params* p, int32_t nch, lbm_storage st, int64_t max_nodes, Sizes& sz) {
    sz = sizes_of(p, nch, max_nodes);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.chan = take(sizeof(Chan) * nch);
    L.seg_ch = take(sizeof(int32_t) * sz.segs);
    L.popA = take(elem_size(st) * Q * 64 * sz.segs);
    L.popB = take(elem_size(st) * Q * 64 * sz.segs);
    L.flags = take(64);
    L.closure = take(sizeof(MlpPacked));
    if (max_nodes > 0) {
        L.node_ch = take(sizeof(int32_t) * max_nodes);
        L.rec = take(sizeof(float) * 20 * max_nodes);
        L.rank = take(sizeof(int32_t) * 27 * max_nodes);
        L.blkbase = take(sizeof(int32_t) * HS * ((max_nodes + 255) / 256));
        // one entry per bin block (256 nodes) or per force workgroup (FS_THREADS / NODE_LANES = 32 nodes)
        L.blkmax = take(sizeof(uint32_t) * ((NODE_LANES * max_nodes + 255) / 256 + 1));
        L.nbase = take(2 * sizeof(int4) * max_nodes);
        for (int k = 0; k < 2; ++k) {
            L.sets[k][0] = take(sizeof(int32_t) * sz.tiles);           // cnt
            L.sets[k][1] = take(sizeof(int32_t) * sz.tiles);           // tile_slot
            L.sets[k][2] = take(sizeof(int32_t) * sz.slots);           // flag_list
            L.sets[k][3] = take(sizeof(int32_t) * sz.slots);           // flag_ch
            L.sets[k][4] = take(sizeof(int32_t) * sz.slots);           // fill
            L.sets[k][5] = take(sizeof(int32_t) * (sz.slots + 1));     // slot_off
            L.sets[k][6] = take(sizeof(IbHdr));                        // header
            L.sets[k][7] = take(sizeof(int32_t) * (sz.slots + 1));     // chunk_off
            L.sets[k][8] = take(sizeof(int32_t) * sz.slots);           // big
        }
        L.list = take(sizeof(int32_t) * sz.list_cap);
        L.force = take(sizeof(float) * 3 * TILE_CELLS * sz.slots);
        L.vel = take(sizeof(float) * 4 * TILE_CELLS * sz.slots);
        L.part = take(sizeof(unsigned long long) * 3 * TILE_CELLS * part_cap_of(sz));
        L.item_slot = take(sizeof(int32_t) * max_items_of(sz));

    }
    L.total = off;
    return L;
}

// Round-up reciprocal for q = (umulhi(n, m) + n) >> s, exact for n < 2^31.
void fast_div(uint32_t d, uint32_t& m, uint32_t& s) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    s = l;
}

lbm_status hip_ok(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_ERR_HIP; }

LatArgs lat_args(lbm_ctx* c) {
    LatArgs a{};
    a.chan = c->d_chan;
    a.seg_ch = c->d_seg_ch;
    a.nseg = c->total_segs;
    a.src = c->pop[c->cur];
    a.dst = c->pop[c->cur ^ 1];
    // every other step walks the lattice backwards: it first reads the cells the previous
    // step wrote last, which the Infinity Cache may still hold
    a.reverse = c->cur & 1;
    if (c->max_nodes > 0) {
        a.tile_slot = c->set[c->ibset].tile_slot;
        a.force = c->d_force;
        a.flag_list = c->set[c->ibset].flag_list;
        a.flag_ch = c->set[c->ibset].flag_ch;
        a.hdr = c->set[c->ibset].hdr;
        a.big = c->set[c->ibset].big;
        a.chunk_off = c->set[c->ibset].chunk_off;
        a.part = c->d_part;
        a.force_w = c->d_force;
    }
    return a;
}

IbArgs ib_args(lbm_ctx* c, int set) {
    IbArgs a{};
    a.chan = c->d_chan;
    a.node_ch = c->d_node_ch;
    a.n = c->n_nodes;
    a.rec = c->d_rec;
    a.set = c->set[set];
    a.other = c->set[set ^ 1];
    a.list = c->d_list;
    a.list_cap = c->list_cap;
    a.force = c->d_force;
    a.vel = c->d_vel;
    a.flags = c->d_flags;
    a.pop = c->pop[c->cur];
    a.kernel = (int32_t)c->kernel;
    a.nch = c->nch;
    a.rank = c->d_rank;
    a.blkbase = c->d_blkbase;
    a.nbin = c->d_nbin;
    a.part = c->d_part;
    a.part_cap = c->part_cap;
    a.item_slot = c->d_item_slot;
    a.blkmax = c->d_blkmax;
    a.blkmax_n = (c->n_nodes + 255) / 256;
    a.max_items = c->max_items;
    a.chunk = SP_CHUNK;
    return a;
}

lbm_status upload_chans(lbm_ctx* c) {
    hipError_t e = hipMemcpyAsync(c->d_chan, c->chans.data(), sizeof(Chan) * c->nch, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return LBM_ERR_HIP;
    return hip_ok(hipStreamSynchronize(c->stream));
}

lbm_status check_ib(lbm_ctx* c, int64_t n) {
    if (c->max_nodes <= 0) return LBM_ERR_STATE;
    if (!c->nodes_set) return LBM_ERR_STATE;
    if (n != c->n_nodes) return LBM_ERR_ARG;
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_status_string(lbm_status s) {
    switch (s) {
        case LBM_OK: return "ok";
        case LBM_ERR_ARG: return "invalid argument";
        case LBM_ERR_STATE: return "call out of order";
        case LBM_ERR_HIP: return "HIP error";
        case LBM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

size_t lbm_workspace_bytes(const lbm_params* ch, int32_t nch, lbm_storage storage, int64_t max_nodes) {
    if (!valid_params(ch, nch) || max_nodes < 0) return 0;
    if (storage != LBM_STORE_F32 && storage != LBM_STORE_F16 && storage != LBM_STORE_BF16) return 0;
    Sizes sz;
    return layout_of(ch, nch, storage, max_nodes, sz).total;
}

lbm_status lbm_create(const lbm_params* ch, int32_t nch, lbm_storage storage, ib_kernel kernel, int64_t max_nodes,
                      void* workspace, size_t bytes, void* stream, lbm_ctx** out) {
    if (!out) return LBM_ERR_ARG;
    *out = nullptr;
    if (!valid_params(ch, nch) || max_nodes < 0 || !workspace) return LBM_ERR_ARG;
    if (storage != LBM_STORE_F32 && storage != LBM_STORE_F16 && storage != LBM_STORE_BF16) return LBM_ERR_ARG;
    if (kernel != IB_PHI_COS4 && kernel != IB_PHI_PESKIN4) return LBM_ERR_ARG;
    if (((uintptr_t)workspace & 255) != 0) return LBM_ERR_ARG;
    if (max_nodes > 0)
        for (int c = 0; c < nch; ++c)
            if (ch[c].nx < 4 || ch[c].nz < 4 || (!ch[c].walls && ch[c].ny < 4)) return LBM_ERR_UNSUPPORTED;
    Sizes sz;
    Layout L = layout_of(ch, nch, storage, max_nodes, sz);
    if (bytes < L.total) return LBM_ERR_ARG;

    lbm_ctx* c = new lbm_ctx();
    c->nch = nch;
    c->storage = storage;
    c->kernel = kernel;
    c->max_nodes = max_nodes;
    c->stream = (hipStream_t)stream;
    c->params.assign(ch, ch + nch);
    for (int q = 0; q < nch; ++q) c->onsite = c->onsite || ch[q].walls == 2;
    c->total_cells = sz.cells;
    c->total_segs = sz.segs;
    c->total_tiles = sz.tiles;
    c->max_slots = sz.slots;
    c->list_cap = sz.list_cap;
    c->esize = elem_size(storage);
    c->ws = (char*)workspace;
    c->lay = L;
    c->d_chan = (Chan*)(c->ws + L.chan);
    c->d_seg_ch = (int32_t*)(c->ws + L.seg_ch);
    c->pop[0] = c->ws + L.popA;
    c->pop[1] = c->ws + L.popB;
    c->d_flags = (uint32_t*)(c->ws + L.flags);
    c->d_mlp = (MlpPacked*)(c->ws + L.closure);
    if (max_nodes > 0) {
        c->d_node_ch = (int32_t*)(c->ws + L.node_ch);
        c->d_rec = (float*)(c->ws + L.rec);
        for (int k = 0; k < 2; ++k) {
            c->set[k].cnt = (int32_t*)(c->ws + L.sets[k][0]);
            c->set[k].tile_slot = (int32_t*)(c->ws + L.sets[k][1]);
            c->set[k].flag_list = (int32_t*)(c->ws + L.sets[k][2]);
            c->set[k].flag_ch = (int32_t*)(c->ws + L.sets[k][3]);
            c->set[k].fill = (int32_t*)(c->ws + L.sets[k][4]);
            c->set[k].slot_off = (int32_t*)(c->ws + L.sets[k][5]);
            c->set[k].hdr = (IbHdr*)(c->ws + L.sets[k][6]);
            c->set[k].chunk_off = (int32_t*)(c->ws + L.sets[k][7]);
            c->set[k].big = (int32_t*)(c->ws + L.sets[k][8]);
        }
        c->d_list = (int32_t*)(c->ws + L.list);
        c->d_rank = (int32_t*)(c->ws + L.rank);
        c->d_blkbase = (int32_t*)(c->ws + L.blkbase);
        c->d_nbin = (int4*)(c->ws + L.nbase);
        c->d_force = (float*)(c->ws + L.force);
        c->d_vel = (float*)(c->ws + L.vel);
        c->d_part = (unsigned long long*)(c->ws + L.part);
        c->part_cap = part_cap_of(sz);
        c->d_item_slot = (int32_t*)(c->ws + L.item_slot);
        c->d_blkmax = (uint32_t*)(c->ws + L.blkmax);
        c->max_items = max_items_of(sz);
    }

    // channel descriptors and the segment map
    c->chans.resize(nch);
    std::vector<int32_t> seg_ch(sz.segs);
    int64_t cell_off = 0, seg_off = 0, tile_off = 0, pop_off = 0, wss_off = 0;
    for (int k = 0; k < nch; ++k) {
        const lbm_params& p = ch[k];
        Chan& d = c->chans[k];
        memset(&d, 0, sizeof(d));
        d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.walls = p.walls;
        d.ncell = (int64_t)p.nx * p.ny * p.nz;
        d.pop_off = pop_off;
        d.cell_off = cell_off;
        d.seg_off = seg_off;
        d.tile_off = tile_off;
        d.wss_off = wss_off;
        d.tnx = (p.nx + TILE - 1) / TILE;
        d.tny = (p.ny + TILE - 1) / TILE;
        d.tnz = (p.nz + TILE - 1) / TILE;
        fast_div((uint32_t)p.nx, d.mx, d.sx);
        fast_div((uint32_t)p.ny, d.my, d.sy);
        d.tau = p.tau;
        d.omega = 1.0f / p.tau;
        d.guo = 1.0f - 0.5f / p.tau;
        for (int q = 0; q < 3; ++q) {
            d.body[q] = p.body_force[q];
            d.uw_lo[q] = p.u_wall_lo[q];
            d.uw_hi[q] = p.u_wall_hi[q];
        }
        const int64_t ns = (d.ncell + 63) / 64;
        for (int64_t s = 0; s < ns; ++s) seg_ch[seg_off + s] = k;
        pop_off += (int64_t)Q * 64 * ns;
        cell_off += d.ncell;
        seg_off += ns;
        tile_off += (int64_t)d.tnx * d.tny * d.tnz;
        wss_off += 2 * (int64_t)p.nx * p.nz;
    }
    hipError_t e = hipMemcpyAsync(c->d_seg_ch, seg_ch.data(), sizeof(int32_t) * sz.segs, hipMemcpyHostToDevice, c->stream);
    lbm_status st = e == hipSuccess ? upload_chans(c) : LBM_ERR_HIP;  // synchronises: seg_ch stays alive
    if (st == LBM_OK) st = hip_ok(launch_fill_i32(c->stream, (int32_t*)c->d_flags, 16, 0));
    if (st == LBM_OK && max_nodes > 0) {
        for (int k = 0; k < 2 && st == LBM_OK; ++k) {
            st = hip_ok(launch_fill_i32(c->stream, c->set[k].cnt, sz.tiles, 0));
            if (st == LBM_OK) st = hip_ok(launch_fill_i32(c->stream, c->set[k].tile_slot, sz.tiles, -1));
            if (st == LBM_OK) st = hip_ok(launch_fill_i32(c->stream, c->set[k].fill, sz.slots, 0));
            if (st == LBM_OK) st = hip_ok(launch_fill_i32(c->stream, c->set[k].slot_off, sz.slots + 1, 0));
            if (st == LBM_OK)
                st = hip_ok(launch_fill_i32(c->stream, (int32_t*)c->set[k].hdr, sizeof(IbHdr) / 4, 0));
            if (st == LBM_OK) st = hip_ok(launch_fill_i32(c->stream, c->set[k].chunk_off, sz.slots + 1, 0));
        }

    }
    if (st == LBM_OK && max_nodes > 0) {
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_state, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_far, hipEventDisableTiming) != hipSuccess)
            st = LBM_ERR_HIP;
    }
    if (st == LBM_OK) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->ib_grid = 4 * (int64_t)cus;
    }
    if (st != LBM_OK) {
        lbm_destroy(c);
        return st;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (c->side) {
        const hipError_t e2 = hipStreamSynchronize(c->side);
        if (e == hipSuccess) e = e2;
        hipStreamDestroy(c->side);
    }
    for (hipEvent_t ev : c->tev) hipEventDestroy(ev);
    if (c->ev_state) hipEventDestroy(c->ev_state);
    if (c->ev_far) hipEventDestroy(c->ev_far);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    delete c;
    return hip_ok(e);
}

lbm_status lbm_init(lbm_ctx* c, const float* rho, const float* u) {
    if (!c) return LBM_ERR_ARG;
    c->bin_age = 0;  // a restart usually puts the nodes back too: bin at the next coupled step
    LatArgs a = lat_args(c);
    a.dst = c->pop[c->cur];
    a.in_rho = rho;
    a.in_u = u;
    return hip_ok(launch_lattice(c, LK_INIT, a));
}

lbm_status lbm_step(lbm_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return LBM_ERR_ARG;
    for (int s = 0; s < nsteps; ++s) {
        LatArgs a = lat_args(c);
        hipError_t e = c->closure ? launch_step_closure(c, a) : launch_lattice(c, LK_STEP, a);
        if (e != hipSuccess) return LBM_ERR_HIP;
        c->cur ^= 1;
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, float* drho, float* v) {
    if (!c) return LBM_ERR_ARG;
    if (!drho && !v) return LBM_OK;
    LatArgs a = lat_args(c);
    a.out_rho = drho;
    a.out_v = v;
    return hip_ok(launch_lattice(c, LK_MOMENTS, a));
}

lbm_status lbm_get_populations(lbm_ctx* c, float* f) {
    if (!c || !f) return LBM_ERR_ARG;
    LatArgs a = lat_args(c);
    a.out_f = f;
    return hip_ok(launch_lattice(c, LK_GETF, a));
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* f) {
    if (!c || !f) return LBM_ERR_ARG;
    LatArgs a = lat_args(c);
    a.dst = c->pop[c->cur];
    a.in_f = f;
    return hip_ok(launch_lattice(c, LK_SETF, a));
}

size_t lbm_state_bytes(const lbm_ctx* c) { return c ? (size_t)Q * 64 * c->total_segs * c->esize : 0; }

lbm_status lbm_get_state(lbm_ctx* c, void* dst) {
    if (!c || !dst) return LBM_ERR_ARG;
    return hip_ok(hipMemcpyAsync(dst, c->pop[c->cur], lbm_state_bytes(c), hipMemcpyDeviceToDevice, c->stream));
}

lbm_status lbm_set_state(lbm_ctx* c, const void* src) {
    if (!c || !src) return LBM_ERR_ARG;
    return hip_ok(hipMemcpyAsync(c->pop[c->cur], src, lbm_state_bytes(c), hipMemcpyDeviceToDevice, c->stream));
}

lbm_status lbm_wall_stress(lbm_ctx* c, float* lo, float* hi) {
    if (!c || !lo || !hi) return LBM_ERR_ARG;
    for (const lbm_params& p : c->params)
        if (!p.walls) return LBM_ERR_STATE;
    LatArgs a = lat_args(c);
    a.out_lo = lo;
    a.out_hi = hi;
    int64_t total = 0;
    for (const lbm_params& p : c->params) total += 2 * (int64_t)p.nx * p.nz;
    return hip_ok(launch_wss(c, a, total));
}

lbm_status lbm_error_flags(lbm_ctx* c, uint32_t* flags) {
    if (!c || !flags) return LBM_ERR_ARG;
    uint32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return LBM_ERR_HIP;
    *flags = h;
    return hip_ok(launch_fill_i32(c->stream, (int32_t*)c->d_flags, 1, 0));
}

lbm_status ib_set_nodes(lbm_ctx* c, int64_t n, const int64_t* node_offsets) {
    if (!c) return LBM_ERR_ARG;
    if (c->max_nodes <= 0) return LBM_ERR_STATE;
    if (n < 0 || n > c->max_nodes) return LBM_ERR_ARG;
    if (!node_offsets && c->nch != 1) return LBM_ERR_ARG;
    std::vector<int64_t> off(c->nch + 1);
    if (node_offsets) {
        for (int k = 0; k <= c->nch; ++k) off[k] = node_offsets[k];
        if (off[0] != 0 || off[c->nch] != n) return LBM_ERR_ARG;
        for (int k = 0; k < c->nch; ++k)
            if (off[k + 1] < off[k]) return LBM_ERR_ARG;
    } else {
        off[0] = 0;
        off[1] = n;
    }
    std::vector<int32_t> node_ch(n > 0 ? n : 1);
    for (int k = 0; k < c->nch; ++k) {
        c->chans[k].node_lo = off[k];
        c->chans[k].node_hi = off[k + 1];
        for (int64_t m = off[k]; m < off[k + 1]; ++m) node_ch[m] = k;
    }
    if (n > 0) {
        hipError_t e = hipMemcpyAsync(c->d_node_ch, node_ch.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return LBM_ERR_HIP;
    }
    lbm_status st = upload_chans(c);  // synchronises, so node_ch may go out of scope
    if (st != LBM_OK) return st;
    c->n_nodes = n;
    c->nodes_set = true;
    c->bin_age = 0;
    return LBM_OK;
}

lbm_status ib_spread(lbm_ctx* c, int64_t n, const double* X, const float* F) {
    if (!c) return LBM_ERR_ARG;
    lbm_status st = check_ib(c, n);
    if (st != LBM_OK) return st;
    if (n > 0 && (!X || !F)) return LBM_ERR_ARG;
    c->ibset ^= 1;
    c->bin_age = 0;  // the coupled steps' lists are replaced
    IbArgs a = ib_args(c, c->ibset);
    a.X = X;
    a.F = F;
    return hip_ok(launch_ib_spread(c, a));
}

lbm_status ib_interp(lbm_ctx* c, int64_t n, const double* X, float* U) {
    if (!c) return LBM_ERR_ARG;
    lbm_status st = check_ib(c, n);
    if (st != LBM_OK) return st;
    if (n > 0 && (!X || !U)) return LBM_ERR_ARG;
    IbArgs a = ib_args(c, c->ibset);
    a.X = X;
    a.U = U;
    return hip_ok(launch_ib_interp(c, a));
}

lbm_status ib_advance(lbm_ctx* c, int64_t n, double* X, const float* U) {
    if (!c || n < 0) return LBM_ERR_ARG;
    if (n > 0 && (!X || !U)) return LBM_ERR_ARG;
    return hip_ok(launch_ib_advance(c->stream, n, X, U));
}

// The constraint arrays of Eq. (4)-(5) are all present when triangles are given, and the FE
// bending arrays of Eq. (6)-(10) when elements are given with a nonzero modulus.
static bool constraints_ok(const ib_membrane* m) {
    if (m->adh_nr < 0 || m->adh_nl < 0) return false;
    if (m->adh_nr > 0) {
        if (m->adh_nl > 0 && (!m->rec_tri || !m->rec_bary || !m->rec_ptr || !m->rec_inc || !m->lig_xz || !m->bond ||
                              !m->lig_count || !m->adh_work))
            return false;
        if (!(m->adh_capture > 0.0) || !(m->adh_nx > 0.0) || !(m->adh_nz > 0.0) || !(m->adh_kT > 0.0)) return false;
        if (m->adh_nx / m->adh_capture > 1e7 || m->adh_nz / m->adh_capture > 1e7) return false;
        if (m->adh_nl > 0 && !m->rec_ptr) return false;
    }
    if (m->elem6 && m->k_fe != 0.0) {
        if (m->ne < 0 || (m->ne > 0 && (!m->elem_ptr || !m->elem_inc || !m->elem_slot || !m->fe_work)))
            return false;
    }
    if (!m->tri) return true;
    if (m->nt < 0 || m->nb < 0 || (m->nt > 0 && m->nb < 1)) return false;
    return m->tri_ptr && m->tri_inc && m->tri_body && m->body_tri && m->rest_area && m->rest_body && m->body_now;
}

lbm_status ib_membrane_rest(const ib_membrane* m, const double* X_rest, void* stream) {
    if (!m || m->n < 0 || (m->n > 0 && !X_rest)) return LBM_ERR_ARG;
    if (!constraints_ok(m)) return LBM_ERR_ARG;
    if (m->nbr_ptr && (!m->nbr_idx || !m->rest_len)) return LBM_ERR_ARG;
    if (m->nh > 0 && (!m->hinges || !m->rest_cs)) return LBM_ERR_ARG;
    if (m->hinge_ptr && m->nh > 0 && !m->hinge_inc) return LBM_ERR_ARG;
    return hip_ok(launch_membrane_rest(m, X_rest, (hipStream_t)stream));
}

lbm_status ib_membrane_forces(const ib_membrane* m, const double* X, float* F, void* stream) {
    if (!m || m->n < 0 || (m->n > 0 && (!X || !F))) return LBM_ERR_ARG;
    if (!constraints_ok(m)) return LBM_ERR_ARG;
    if (m->nbr_ptr && (!m->nbr_idx || !m->rest_len)) return LBM_ERR_ARG;
    if (m->hinge_ptr && (!m->hinge_inc || !m->hinges || !m->rest_cs)) return LBM_ERR_ARG;
    return hip_ok(launch_membrane_forces(m, X, F, (hipStream_t)stream));
}

int64_t ib_adhesion_work_ints(int64_t nl, double nx, double nz, double capture) {
    if (nl < 0 || !(nx > 0.0) || !(nz > 0.0) || !(capture > 0.0) || nx / capture > 1e7 || nz / capture > 1e7) return 0;
    return adhesion_work_ints(nl, nx, nz, capture);
}

lbm_status ib_adhesion_step(const ib_membrane* m, const double* X, void* stream) {
    if (!m || !X || !constraints_ok(m) || !adhesion_on(*m)) return LBM_ERR_ARG;
    return hip_ok(launch_adhesion_step(m, X, nullptr, (hipStream_t)stream));
}

// Lattice update of the whole context with the body force alone, on the second stream,
// once the state it reads is complete on the main stream.
static hipError_t far_update(lbm_ctx* c) {
    hipError_t e = hipEventRecord(c->ev_state, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_state, 0);
    if (e != hipSuccess) return e;
    LatArgs la = lat_args(c);
    la.tile_slot = nullptr;
    la.force = nullptr;
    hipStream_t main = c->stream;
    c->stream = c->side;
    e = launch_lattice(c, LK_STEP, la);
    c->stream = main;
    if (e == hipSuccess) e = hipEventRecord(c->ev_far, c->side);
    return e;
}

// Fig. 1, `nsteps` times: forces -> spread -> lattice update -> interpolation (+ move).
// With the overlapped schedule, the update of step s+1 away from the IB tiles (body force
// only) is issued on the second stream right after step s's update, so it runs during the
// interpolation of step s and the force / spread pipeline of step s+1; step s+1 then waits
// for it and updates the flagged tiles' cells with their force.  Both buffers are only
// read by everything that runs concurrently with the far update except its own output.
static lbm_status coupled(lbm_ctx* c, const ib_membrane* m, int32_t nsteps, double* X, float* F, float* U) {
    const bool ov = c->launch.overlap && c->side && !c->closure && nsteps > 0;
    if (ov && far_update(c) != hipSuccess) return LBM_ERR_HIP;
    // with a membrane and rebin > 1 the nodes are binned (with a margin) every `rebin` steps
    const int rebin = m ? c->launch.rebin : 1;
    for (int s = 0; s < nsteps; ++s) {
        const bool bin = rebin <= 1 || c->bin_age == 0;
        if (bin) c->ibset ^= 1;
        IbArgs a = ib_args(c, c->ibset);
        a.X = X;
        a.F = F;
        if (rebin > 1) {
            a.margin = REBIN_MARGIN;
            a.scale_local = 1;
        }
        // Without the closure or the second stream, the lattice update away from the IB tiles
        // (body force only) runs in the spread's launch, and the flagged tiles' cells are then
        // updated with their force (merging split tiles' partial sums on the way): bitwise the
        // fused update.
        const bool split_update =
            m && !ov && !c->closure && (c->launch.split == 1 || (c->launch.split == -1 && c->nch == 1));
        // longer spread work items only where the lattice update is long enough to hide them
        if (split_update && c->total_cells >= SP_SPLIT_MIN_CELLS) a.chunk = SP_CHUNK_SPLIT;
        if (m) {
            // the binning and the scan need only X: they run beside the hinge and node forces,
            // and the force kernel fills in what the spread needs of F
            if (launch_forces_scatter(c, m, X, F, a, bin) != hipSuccess) return LBM_ERR_HIP;
            if (!split_update && launch_ib_spread_items(c, a) != hipSuccess) return LBM_ERR_HIP;
        } else if (launch_ib_spread(c, a) != hipSuccess) {
            return LBM_ERR_HIP;
        }
        LatArgs la = lat_args(c);
        hipError_t e;
        // the launch timer brackets the launch that updates the lattice (eager calls only)
        const bool timed = c->timer && !c->capturing && !ov && c->tcount < LBM_TIMER_PAIRS;
        if (timed && hipEventRecord(c->tev[2 * c->tcount], c->stream) != hipSuccess) return LBM_ERR_HIP;
        if (split_update) {
            e = launch_spread_far(c, a, la);
            if (timed && e == hipSuccess) e = hipEventRecord(c->tev[2 * c->tcount + 1], c->stream);
            if (e == hipSuccess) e = launch_step_tiles(c, la, true);
        } else if (ov) {
            e = hipStreamWaitEvent(c->stream, c->ev_far, 0);
            if (e == hipSuccess) e = launch_step_tiles(c, la);
        } else {
            e = c->closure ? launch_step_closure(c, la) : launch_lattice(c, LK_STEP, la);
            if (timed && e == hipSuccess) e = hipEventRecord(c->tev[2 * c->tcount + 1], c->stream);
        }
        if (timed) {
            c->tkind = split_update ? 1 : (c->closure ? 2 : 0);
            ++c->tcount;
        }
        if (e != hipSuccess) return LBM_ERR_HIP;
        c->cur ^= 1;
        if (ov && s + 1 < nsteps && far_update(c) != hipSuccess) return LBM_ERR_HIP;
        IbArgs b = ib_args(c, c->ibset);
        b.X = X;
        b.U = U;
        b.Xout = X;  // X <- X + U, fused into the gather
        b.use_rec = 1;  // X is the spread's X
        if (launch_ib_interp(c, b) != hipSuccess) return LBM_ERR_HIP;
        // the adhesion's Monte-Carlo step at the moved positions (the last box of Fig. 1)
        if (m && launch_adhesion_step(m, X, (uint32_t*)c->d_flags, c->stream) != hipSuccess) return LBM_ERR_HIP;
        c->bin_age = rebin > 1 ? (c->bin_age + 1) % rebin : 0;
    }
    return LBM_OK;
}

lbm_status lbm_coupled_steps(lbm_ctx* c, const ib_membrane* m, int32_t nsteps, double* X, float* F, float* U) {
    if (!c || nsteps < 0) return LBM_ERR_ARG;
    lbm_status st = check_ib(c, c->n_nodes);
    if (st != LBM_OK) return st;
    if (c->n_nodes > 0 && (!X || !F || !U)) return LBM_ERR_ARG;
    if (m && (m->n != c->n_nodes || !constraints_ok(m))) return LBM_ERR_ARG;
    return coupled(c, m, nsteps, X, F, U);
}

lbm_status lbm_graph_capture(lbm_ctx* c, const ib_membrane* m, int32_t nsteps, double* X, float* F, float* U) {
    if (!c || nsteps < 2 || (nsteps & 1)) return LBM_ERR_ARG;
    // a replay must end at the binning phase and tile set it started from
    if (m && c->launch.rebin > 1 && nsteps % (2 * c->launch.rebin)) return LBM_ERR_ARG;
    lbm_status st = check_ib(c, c->n_nodes);
    if (st != LBM_OK) return st;
    if (c->n_nodes > 0 && (!X || !F || !U)) return LBM_ERR_ARG;
    if (m && (m->n != c->n_nodes || !constraints_ok(m))) return LBM_ERR_ARG;
    if (c->gexec) { hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (c->graph) { hipGraphDestroy(c->graph); c->graph = nullptr; }
    const int cur0 = c->cur, set0 = c->ibset, age0 = c->bin_age;
    if (c->stream == nullptr) return LBM_ERR_UNSUPPORTED;  // the legacy default stream cannot be captured
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_ERR_HIP;
    c->capturing = true;
    st = coupled(c, m, nsteps, X, F, U);
    c->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    // nothing ran during capture; with an even step count the buffer and tile-set
    // parities are back where they started when a replay ends
    c->cur = cur0;
    c->ibset = set0;
    c->bin_age = age0;
    if (st != LBM_OK || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return st != LBM_OK ? st : LBM_ERR_HIP;
    }
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return LBM_ERR_HIP;
    }
    c->graph = g;
    c->graph_cur = cur0;
    c->graph_set = set0;
    c->graph_age = age0;
    return LBM_OK;
}

lbm_status lbm_graph_launch(lbm_ctx* c, int32_t repeats) {
    if (!c || repeats < 0) return LBM_ERR_ARG;
    if (!c->gexec) return LBM_ERR_STATE;
    // the graph's kernels read and write the buffers and tile sets of the parities it was
    // captured at: an odd number of eager steps (or a lone lbm_step / ib_spread) since then
    // would make it replay from stale state
    if (c->cur != c->graph_cur || c->ibset != c->graph_set || c->bin_age != c->graph_age) return LBM_ERR_STATE;
    for (int r = 0; r < repeats; ++r)
        if (hipGraphLaunch(c->gexec, c->stream) != hipSuccess) return LBM_ERR_HIP;
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* c, const lbm_launch* cfg) {
    if (!c || !cfg) return LBM_ERR_ARG;
    const int b = cfg->block;
    if (b != 64 && b != 128 && b != 256 && b != 512 && b != 1024) return LBM_ERR_ARG;
    if (cfg->persistent < 0 || (cfg->xcd_remap != 0 && cfg->xcd_remap != 1) ||
        (cfg->nontemporal != 0 && cfg->nontemporal != 1) || cfg->vec < 0 || cfg->vec > 4 || cfg->vec == 3 ||
        (cfg->overlap != 0 && cfg->overlap != 1) || cfg->split < -1 || cfg->split > 1 || cfg->rebin < 1 ||
        cfg->rebin > 64)
        return LBM_ERR_ARG;
    c->launch = *cfg;
    c->bin_age = 0;  // bin at the next coupled step
    return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_ctx* c, lbm_launch* cfg) {
    if (!c || !cfg) return LBM_ERR_ARG;
    *cfg = c->launch;
    return LBM_OK;
}

lbm_status lbm_launch_timer(lbm_ctx* c, int32_t enable) {
    if (!c || (enable != 0 && enable != 1)) return LBM_ERR_ARG;
    if (enable && c->tev.empty()) {
        // timing-only events: without the system-scope fence at each record, which would add
        // the writeback of the L2 that the timed launch left dirty to its measured time
        std::vector<hipEvent_t> evs(2 * LBM_TIMER_PAIRS, nullptr);
        for (hipEvent_t& ev : evs)
            if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) {
                for (hipEvent_t made : evs)
                    if (made) hipEventDestroy(made);
                return LBM_ERR_HIP;
            }
        c->tev.swap(evs);
    }
    c->timer = enable != 0;
    c->tcount = 0;
    c->tkind = -1;
    return LBM_OK;
}

lbm_status lbm_launch_timer_read(lbm_ctx* c, int64_t* count, double* mean_us, int32_t* kind) {
    if (!c || !count || !mean_us) return LBM_ERR_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_ERR_HIP;
    double tot = 0.0;
    for (int64_t k = 0; k < c->tcount; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]) != hipSuccess) return LBM_ERR_HIP;
        tot += ms;
    }
    *count = c->tcount;
    *mean_us = c->tcount ? 1e3 * tot / (double)c->tcount : 0.0;
    if (kind) *kind = c->tkind;
    c->tcount = 0;
    c->tkind = -1;
    return LBM_OK;
}

lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, int32_t variant, int64_t grid, void* stream) {
    if (!src || !dst || (bytes & 15) || variant < 0 || variant > 1 || grid < 0) return LBM_ERR_ARG;
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return LBM_ERR_ARG;
    return hip_ok(launch_copy16((hipStream_t)stream, src, dst, (int64_t)bytes, variant, grid));
}

// ---------------------------------------------------------------- learned closure
}  // extern "C"
namespace {
constexpr int64_t MLP_GRID = 1024;  // fixed workgroup counts: results do not depend on the GPU
constexpr int64_t NORM_GRID = 1024;

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
}  // namespace
extern "C" {

lbm_status mlp_pack(const float* params, const float* norm, float c_guard, void* packed, void* stream) {
    if (!params || !norm || !packed || !(c_guard >= 0.0f) || !aligned16(packed)) return LBM_ERR_ARG;
    return hip_ok(launch_mlp_pack((hipStream_t)stream, params, norm, c_guard, (MlpPacked*)packed));
}

lbm_status lbm_set_closure(lbm_ctx* c, const float* params, const float* norm, float c_guard, int32_t enable) {
    if (!c) return LBM_ERR_ARG;
    if (!enable) {
        c->closure = false;
        return LBM_OK;
    }
    lbm_status st = mlp_pack(params, norm, c_guard, c->d_mlp, c->stream);
    if (st == LBM_OK) c->closure = true;
    return st;
}

lbm_status lbm_closure_guarded(lbm_ctx* c, uint64_t* count) {
    if (!c || !count) return LBM_ERR_ARG;
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->d_flags + 2, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return LBM_ERR_HIP;
    *count = (uint64_t)h;
    return hip_ok(launch_fill_i32(c->stream, (int32_t*)(c->d_flags + 2), 2, 0));
}

lbm_status mlp_forward(const void* packed, const float* raw, int64_t B, float* dm, void* stream) {
    if (!packed || B < 0 || (B > 0 && (!raw || !dm))) return LBM_ERR_ARG;
    if (!aligned16(packed)) return LBM_ERR_ARG;
    return hip_ok(launch_mlp_forward((hipStream_t)stream, (const MlpPacked*)packed, raw, B, dm, MLP_GRID));
}

size_t mlp_grad_workspace_bytes(int64_t B) {
    if (B < 1) return 0;
    return (size_t)mlp_grad_blocks(B, MLP_GRID) * (MLP_PARAMS + 1) * sizeof(float);
}

lbm_status mlp_grad(const void* packed, const float* raw, const float* target, int64_t B, float* grad, float* loss,
                    void* work, size_t work_bytes, void* stream) {
    if (!packed || !raw || !target || !grad || !work || B < 1 || !aligned16(packed)) return LBM_ERR_ARG;
    if (work_bytes < mlp_grad_workspace_bytes(B)) return LBM_ERR_ARG;
    const int64_t nblk = mlp_grad_blocks(B, MLP_GRID);
    return hip_ok(launch_mlp_grad((hipStream_t)stream, (const MlpPacked*)packed, raw, target, B, (float*)work, nblk,
                                  grad, loss));
}

// ---------------------------------------------------------------- mlp_grad without allocation
}  // extern "C"
namespace {
// Scratch of mlp_grad_noalloc: the partial row (MLP_PARAMS gradient entries + the loss) of each
// k_mlp_grad workgroup, as many rows as that kernel ever has workgroups (MLP_GRID), so the
// variant partitions every B exactly as mlp_grad does.  k_mlp_grad writes every entry of its
// rows before k_grad_reduce reads them, so nothing needs clearing between calls.  Each GPU holds
// its own copy (MLP_GRID * 6289 floats = 25.8 MB) until the process ends.  In host code the
// array's name stands for a host-side shadow: only the address looked up per device is used.
constexpr int64_t NOALLOC_ROWS = MLP_GRID;
static __device__ __align__(256) float scratch[NOALLOC_ROWS * (MLP_PARAMS + 1)];

constexpr int NOALLOC_MAX_DEVICES = 256;
std::mutex noalloc_mu;
float* noalloc_ptr[NOALLOC_MAX_DEVICES];  // device address of each GPU's scratch, once looked up

// The device address of the current GPU's scratch (looked up on the first call on that GPU).
lbm_status noalloc_scratch(int dev, float** out) {
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_ERR_HIP;
        noalloc_ptr[dev] = (float*)p;
    }
    *out = noalloc_ptr[dev];
    return LBM_OK;
}
}  // namespace
extern "C" {

lbm_status mlp_grad_noalloc(const void* packed, const float* raw, const float* target, int64_t B, float* grad,
                            float* loss, void* stream) {
    if (!packed || !raw || !target || !grad || B < 1 || !aligned16(packed)) return LBM_ERR_ARG;
    const int64_t nblk = mlp_grad_blocks(B, MLP_GRID);
    if (nblk > NOALLOC_ROWS) return LBM_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LBM_ERR_HIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LBM_ERR_UNSUPPORTED;
    if (stream) {
        hipDevice_t sdev = -1;
        if (hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess) return LBM_ERR_HIP;
        if (sdev != dev) return LBM_ERR_ARG;  // the scratch looked up is the current GPU's
    }
    float* work = nullptr;
    lbm_status st = noalloc_scratch(dev, &work);
    if (st != LBM_OK) return st;
    return hip_ok(launch_mlp_grad((hipStream_t)stream, (const MlpPacked*)packed, raw, target, B, work, nblk, grad,
                                  loss));
}

lbm_status mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v || n < 0 || step < 1) return LBM_ERR_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) return LBM_ERR_ARG;
    if (n == 0) return LBM_OK;
    return hip_ok(launch_adam((hipStream_t)stream, params, grad, m, v, n, step, lr, beta1, beta2, eps));
}

static int64_t norm_blocks(int64_t B) {
    const int64_t nb = (B + 15) / 16;
    return nb < NORM_GRID ? nb : NORM_GRID;
}

size_t mlp_norm_workspace_bytes(int64_t B) { return B < 1 ? 0 : (size_t)norm_blocks(B) * 48 * sizeof(double); }

lbm_status mlp_norm(const float* raw, const float* target, int64_t B, float* norm, void* work, size_t work_bytes,
                    void* stream) {
    if (!raw || !target || !norm || !work || B < 1) return LBM_ERR_ARG;
    if (work_bytes < mlp_norm_workspace_bytes(B)) return LBM_ERR_ARG;
    return hip_ok(launch_norm((hipStream_t)stream, raw, target, B, (double*)work, (int)norm_blocks(B), norm));
}

lbm_status lbm_restrict(lbm_ctx* c, float tau_coarse, float* g_c, float* F_c) {
    if (!c || !g_c || !F_c || !(tau_coarse > 0.5f)) return LBM_ERR_ARG;
    if (c->nch != 1) return LBM_ERR_UNSUPPORTED;
    const lbm_params& p = c->params[0];
    if ((p.nx & 1) || (p.ny & 1) || (p.nz & 1)) return LBM_ERR_UNSUPPORTED;
    if (p.walls == 2) return LBM_ERR_UNSUPPORTED;  // 2x2x2 blocks align with halfway walls only
    LatArgs a = lat_args(c);
    return hip_ok(launch_restrict(c, a, 2.0f * tau_coarse / p.tau, g_c, F_c));
}

lbm_status closure_targets(const lbm_params* coarse, const float* g0, const float* F, const float* g1, float* feat,
                           float* target, void* stream) {
    if (!valid_params(coarse, 1) || !g0 || !F || !g1 || !feat || !target) return LBM_ERR_ARG;
    if (coarse->walls == 2) return LBM_ERR_UNSUPPORTED;  // coarse-graining assumes halfway walls
    Chan ch;
    memset(&ch, 0, sizeof(ch));
    ch.nx = coarse->nx;
    ch.ny = coarse->ny;
    ch.nz = coarse->nz;
    ch.walls = coarse->walls;
    ch.ncell = (int64_t)coarse->nx * coarse->ny * coarse->nz;
    fast_div((uint32_t)ch.nx, ch.mx, ch.sx);
    fast_div((uint32_t)ch.ny, ch.my, ch.sy);
    ch.tau = coarse->tau;
    ch.omega = 1.0f / coarse->tau;
    ch.guo = 1.0f - 0.5f / coarse->tau;
    for (int q = 0; q < 3; ++q) {
        ch.body[q] = coarse->body_force[q];
        ch.uw_lo[q] = coarse->u_wall_lo[q];
        ch.uw_hi[q] = coarse->u_wall_hi[q];
    }
    return hip_ok(launch_targets((hipStream_t)stream, ch, g0, F, g1, feat, target));
}

}  // extern "C"
