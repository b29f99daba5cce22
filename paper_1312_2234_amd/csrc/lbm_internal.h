// lbm_internal.h -- host-side context and the launchers shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lbm.h"
#include "lbm_device.h"

namespace lbmib {

// Header of one immersed-boundary tile set (device).
struct IbHdr {
    int32_t nflag;       // flagged tiles of the last spread using this set
    uint32_t fmax_bits;  // max |F| over the nodes (float bits)
    int32_t scale_exp;   // fixed-point scale 2^scale_exp of the spread accumulation
    int32_t nonfinite;   // 1 if a force was Inf/NaN
    int32_t nchunk;      // spread work items (node-list chunks) of the flagged tiles
    int32_t pad[3];
};

// Device arrays of one tile set.  Two sets alternate between successive spreads so
// that each spread can clear the set used two spreads earlier without an extra launch.
struct IbSet {
    int32_t* cnt;        // [ntiles] nodes whose stencil touches the tile
    int32_t* tile_slot;  // [ntiles] slot of a flagged tile, -1 otherwise
    int32_t* flag_list;  // [max_slots] tile id of each slot
    int32_t* flag_ch;    // [max_slots] channel of each slot
    int32_t* fill;       // [max_slots] fill counters of the node lists
    int32_t* slot_off;   // [max_slots+1] list offsets
    int32_t* chunk_off;  // [max_slots+1] first spread work item of each slot
    int32_t* big;        // [max_slots] first partial block of a slot split into several work
                         // items, -1 if the slot is one work item
    IbHdr* hdr;
};

// Spreading splits a tile's node list into chunks of SP_CHUNK nodes; each chunk of a split
// tile stores its exact fixed-point partial sums in one of `part_cap` partial blocks, and a
// merge kernel adds them up.
// The kernels that walk the flagged tiles cell by cell (flagged-tile update, velocity blocks)
// give each tile TILE_PARTS workgroups of TILE_CELLS / TILE_PARTS threads (one wavefront
// each): a few hundred tiles then spread over every CU and XCD.  Measured on the shear
// channel's 219 tiles, tile update / velocity blocks: 1 part 14.0 / 10.3 us, 2 parts
// 13.3 / 9.9, 4 parts 12.4 / 9.5, 8 parts 10.3 / 8.9.
constexpr int TILE_PARTS = 8;
constexpr int SP_CHUNK = 256;
// Chunk of the split coupled step: there the spread runs hidden under the lattice update, and
// fewer split tiles leave less merging to the flagged-tile update (results are the same exact
// integer sums whatever the chunking).  Capacities are sized for SP_CHUNK, the smaller one.
constexpr int SP_CHUNK_SPLIT = 1024;
// ... used from this many cells on: on the 0.5 M-cell coarse twin the update (15 us) cannot
// hide the longer items (step 77.5 -> 99.2 us), on the 4.2 M-cell shear channel it can
// (185.6 -> 182.3 us)
constexpr int64_t SP_SPLIT_MIN_CELLS = int64_t(1) << 21;
// Binning: per-block LDS hash of tile counts (HS entries).
constexpr int HS_BITS = 9;
constexpr int HS = 1 << HS_BITS;
constexpr int64_t SP_PART_MAX = 16384;

// Arguments of the lattice kernels (walk over 64-cell segments of all channels).
struct LatArgs {
    const Chan* chan;
    const int32_t* seg_ch;
    int64_t nseg;
    const void* src;        // current stored (post-collision, shifted) populations
    void* dst;              // next buffer (lbm_step) or unused
    const int32_t* tile_slot;  // IB tile -> slot of the current force field, or null
    const float* force;        // [slots][3][512]
    const int32_t* flag_list;  // flagged tiles of the current force field (tile update)
    const int32_t* flag_ch;
    const IbHdr* hdr;
    const int32_t* big;        // first partial block of each split slot, -1 otherwise
    const int32_t* chunk_off;  // [slots+1] work items of each slot
    const unsigned long long* part;  // fixed-point partial blocks of split slots
    float* force_w;            // force blocks, written by the merging tile update
    int32_t remap;          // XCD-aware block order
    int32_t persistent;     // loop over blocks
    int32_t reverse;        // walk the segments from the last one (every other step)
    // auxiliary inputs / outputs of the non-step kernels
    const float* in_rho;
    const float* in_u;
    const float* in_f;
    float* out_rho;
    float* out_v;
    float* out_f;
    float* out_lo;
    float* out_hi;
};

struct IbArgs {
    const Chan* chan;
    const int32_t* node_ch;
    int64_t n;
    const double* X;
    const float* F;
    float* U;
    double* Xout;
    float* rec;             // [n][20] node records
    IbSet set;              // tile set of this spread
    IbSet other;            // set cleared by this spread
    int32_t* list;
    int64_t list_cap;
    float* force;           // [max_slots][3][512]
    float* vel;             // [max_slots][3][512]
    uint32_t* flags;
    const void* pop;        // current stored populations (interpolation)
    int32_t kernel;         // ib_kernel
    int32_t use_rec;        // interpolation at the positions of the latest spread: reuse its node records
    int32_t nch;
    int32_t* rank;          // [n][27] packed rank of a node in each tile list it joins
    int32_t* blkbase;       // [ceil(n/256)][HS] per-block base of each hashed tile
    int4* nbin;             // [n][2] with a binning margin: floor(X - margin) and floor(X + margin)
                            // per axis at the node's last binning (x, y, z; w unused)
    double margin;          // binning margin (lattice units); 0 = the exact stencil
    int32_t scale_local;    // the spread's work items reduce the force maximum themselves
    int32_t rec_in_forces;  // the membrane-force kernel writes the nodes' stencil bases and weights
    int32_t do_scan;        // the scan workgroup of the force launch runs (binning steps)
    unsigned long long* part;  // [part_cap][3][512] fixed-point partial sums of split tiles' chunks
    int64_t part_cap;
    uint32_t* blkmax;       // max |F| (float bits) per bin block, or per membrane-force workgroup
    int64_t blkmax_n;       // entries of blkmax reduced for the spread's scale
    int32_t scale_in_scatter;  // the scatter's first workgroup sets the scale (not the scan)
    int32_t* item_slot;     // [max_items] slot of each spread work item
    int64_t max_items;
    int32_t chunk;          // nodes per spread work item: SP_CHUNK, or SP_CHUNK_SPLIT
};

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t per = G >> 3, rem = G & 7, x = b & 7;
    return x * per + (x < rem ? x : rem) + (b >> 3);
}

// Iterate the segments assigned to this wavefront; body(ch, n) runs for every valid cell.
template <class Body>
__device__ __forceinline__ void for_cells(const LatArgs& a, Body body) {
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t G = gridDim.x;
    int64_t L = a.remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    for (;; L += G) {
        const int64_t sw = L * wpb + wave;
        if (sw >= a.nseg) break;
        const int64_t seg = a.reverse ? a.nseg - 1 - sw : sw;
        const int c = a.seg_ch[seg];
        const Chan& ch = a.chan[c];
        const int64_t n = (seg - ch.seg_off) * 64 + lane;
        if (n < ch.ncell) body(ch, (int32_t)n);
        if (!a.persistent) break;
    }
}

__device__ __forceinline__ void ib_force(const LatArgs& a, const Chan& ch, int x, int y, int z, float& Fx,
                                         float& Fy, float& Fz) {
    Fx = ch.body[0];
    Fy = ch.body[1];
    Fz = ch.body[2];
    if (a.tile_slot) {
        const int slot = a.tile_slot[tile_of(ch, x, y, z)];
        if (slot >= 0) {
            const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS) + tile_local(x, y, z);
            Fx += fb[0];
            Fy += fb[TILE_CELLS];
            Fz += fb[2 * TILE_CELLS];
        }
    }
}

// Packed learned-closure network (device): BF16 weight fragments in the matrix-core
// operand order, FP32 biases and the input / output scaling.
constexpr int MLP_NIN = 16, MLP_NH = 64, MLP_NOUT = 16, MLP_NNC = 15;
constexpr int MLP_NFRAG = 24;      // forward: 4 (16x64) + 16 (64x64) + 4 (64x16) tiles of 16x16
constexpr int MLP_NFRAG_ALL = 44;  // + backward: 4 (W3) + 16 (W2) transposed tiles
struct MlpPacked {
    uint16_t frag[MLP_NFRAG_ALL][64][4];  // lane-major A operands, 4 bf16 per lane
    float bias[MLP_NH + MLP_NH + MLP_NOUT];
    float norm[3 * MLP_NIN];          // in_mean[16], in_scale[16], out_scale[16]
    float c_guard;
    float pad[15];
};
static_assert(sizeof(MlpPacked) == MLP_PACKED_BYTES, "packed network size");

struct Layout {
    size_t chan, seg_ch, popA, popB, flags, closure, node_ch, rec, rank, blkbase, nbase, sets[2][9], list, force,
        vel, part, item_slot, blkmax, total;
};

}  // namespace lbmib

struct lbm_ctx {
    int nch = 0;
    lbm_storage storage = LBM_STORE_F32;
    bool onsite = false;  // some channel has on-site walls (walls = 2)
    ib_kernel kernel = IB_PHI_COS4;
    int64_t max_nodes = 0;
    hipStream_t stream = nullptr;
    std::vector<lbm_params> params;
    std::vector<lbmib::Chan> chans;
    int64_t total_cells = 0, total_segs = 0, total_tiles = 0, max_slots = 0, list_cap = 0;
    size_t esize = 4;
    char* ws = nullptr;
    lbmib::Layout lay{};
    lbmib::Chan* d_chan = nullptr;
    int32_t* d_seg_ch = nullptr;
    void* pop[2] = {nullptr, nullptr};
    int cur = 0;  // buffer holding the current state
    uint32_t* d_flags = nullptr;
    // immersed boundary
    int64_t n_nodes = 0;
    bool nodes_set = false;
    int32_t* d_node_ch = nullptr;
    float* d_rec = nullptr;
    lbmib::IbSet set[2]{};
    int ibset = 0;  // set of the latest spread (both clean at creation)
    int32_t* d_list = nullptr;
    int32_t* d_rank = nullptr;
    int32_t* d_blkbase = nullptr;
    int4* d_nbin = nullptr;
    unsigned long long* d_part = nullptr;
    int64_t part_cap = 0;
    int32_t* d_item_slot = nullptr;
    uint32_t* d_blkmax = nullptr;
    int64_t max_items = 0;
    int64_t ib_grid = 1024;  // workgroups of the grid-stride IB kernels (set from the CU count)
    float* d_force = nullptr;
    float* d_vel = nullptr;
    lbm_launch launch{256, 1, 0, 1, 0, 0, -1, 1};
    int bin_age = 0;  // coupled steps since the last binning (rebin > 1); 0 = bin at the next step
    hipStream_t side = nullptr;         // second stream of the overlapped coupled step
    hipEvent_t ev_state = nullptr, ev_far = nullptr;
    lbmib::MlpPacked* d_mlp = nullptr;
    bool closure = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // buffer and tile-set parities the captured graph was recorded at (it reads and writes
    // fixed buffers, so it may only be replayed from the same parities)
    int graph_cur = 0, graph_set = 0, graph_age = 0;
    bool capturing = false;  // inside lbm_graph_capture
    // launch timer (measurement helper): event pairs around the lattice-update launches of eager
    // coupled steps
    bool timer = false;
    std::vector<hipEvent_t> tev;
    int64_t tcount = 0;
    int32_t tkind = -1;
};

namespace lbmib {

// lattice.hip
hipError_t launch_lattice(lbm_ctx* c, int which, const LatArgs& a);
hipError_t launch_step_tiles(lbm_ctx* c, const LatArgs& a, bool merge = false);
enum { LK_STEP = 0, LK_INIT, LK_MOMENTS, LK_GETF, LK_SETF, LK_WSS };
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
hipError_t launch_wss(lbm_ctx* c, const LatArgs& a, int64_t total);
hipError_t launch_copy16(hipStream_t s, const void* src, void* dst, int64_t bytes, int variant, int64_t grid);

// ib.hip
hipError_t launch_ib_spread(lbm_ctx* c, const IbArgs& a);
hipError_t launch_ib_spread_binned(lbm_ctx* c, const IbArgs& a);
hipError_t launch_ib_spread_items(lbm_ctx* c, const IbArgs& a);
hipError_t launch_ib_interp(lbm_ctx* c, const IbArgs& a);
hipError_t launch_ib_advance(hipStream_t s, int64_t n, double* X, const float* U);
hipError_t launch_membrane_rest(const ib_membrane* m, const double* X_rest, hipStream_t s);
hipError_t launch_membrane_forces(const ib_membrane* m, const double* X, float* F, hipStream_t s);
hipError_t launch_forces_scatter(lbm_ctx* c, const ib_membrane* m, const double* X, float* F, IbArgs& a, bool bin);
// binning margin of the rebin mode (lattice units)
constexpr double REBIN_MARGIN = 0.5;
// Lanes per node of the membrane-force kernels (measured on the shear channel, force launch
// with node-centric hinges: 8 lanes 16.4 us, 16 lanes 26 us).
constexpr int NODE_LANES = 8;
// adhesion (adhesion.hip)
bool adhesion_on(const ib_membrane& m);
int64_t adhesion_work_ints(int64_t nl, double nx, double nz, double capture);
hipError_t launch_adhesion_setup(const ib_membrane* m, hipStream_t s);
hipError_t launch_adhesion_step(const ib_membrane* m, const double* X, uint32_t* flags, hipStream_t s);
hipError_t launch_spread_far(lbm_ctx* c, const IbArgs& a, const LatArgs& la);

// closure.hip
hipError_t launch_mlp_pack(hipStream_t s, const float* params, const float* norm, float c_guard, MlpPacked* P);
hipError_t launch_step_closure(lbm_ctx* c, const LatArgs& a);
hipError_t launch_mlp_forward(hipStream_t s, const MlpPacked* P, const float* raw, int64_t B, float* dm,
                              int64_t grid_max);
int64_t mlp_grad_blocks(int64_t B, int64_t grid_max);
hipError_t launch_mlp_grad(hipStream_t s, const MlpPacked* P, const float* raw, const float* tgt, int64_t B,
                           float* partial, int64_t nblk, float* grad, float* loss);
hipError_t launch_adam(hipStream_t s, float* th, const float* g, float* m, float* v, int64_t n, int step, float lr,
                       float b1, float b2, float eps);
hipError_t launch_norm(hipStream_t s, const float* raw, const float* tgt, int64_t B, double* part, int nblk,
                       float* norm);
hipError_t launch_restrict(lbm_ctx* c, const LatArgs& a, float resc, float* gc, float* Fc);
hipError_t launch_targets(hipStream_t s, const Chan& ch, const float* g0, const float* F, const float* g1,
                          float* feat, float* target);

// Calls f(St{}) with the storage form of the context: StF32 / StF16 / StBF16, wrapped in
// OnSite<> when a channel has on-site walls, so that only such contexts run kernels with the
// wall-row branch compiled in.  Every branch of f must return the same type.
template <class F>
auto with_storage(const lbm_ctx* c, F&& f) {
    if (c->onsite) {
        switch (c->storage) {
            case LBM_STORE_F16: return f(OnSite<StF16>{});
            case LBM_STORE_BF16: return f(OnSite<StBF16>{});
            default: return f(OnSite<StF32>{});
        }
    }
    switch (c->storage) {
        case LBM_STORE_F16: return f(StF16{});
        case LBM_STORE_BF16: return f(StBF16{});
        default: return f(StF32{});
    }
}

}  // namespace lbmib
