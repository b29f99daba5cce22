// ib.hip -- immersed-boundary coupling (section 3.4.2, Eq. (33)-(36)) and membrane forces
// (section 3.1, Eq. (2)-(3) and a dihedral bending stand-in) for gfx950.
//
// Spreading (Eq. (34)) is organised around 8x8x8 lattice tiles instead of the paper's
// one-thread-per-lattice-node launch:
//   bin      one thread per node: stencil base, the 3x4 kernel weights, the tiles its
//            4x4x4 stencil touches (count per tile; first toucher appends the tile to the
//            flagged list), max |F|;
//   scan     one workgroup: list offsets of the flagged tiles, tile -> slot map; clears
//            the tile set of the spread before last;
//   scatter  one thread per node: its id into the list of every tile it touches;
//   spread   one workgroup per flagged tile: the tile's nodes add their stencil
//            contributions into a 512-cell LDS accumulator, then the tile's force block
//            is written.
// The LDS accumulation is 64-bit fixed point with a per-call scale from max |F|, so the
// sum is exact and independent of the order in which nodes arrive: the result is
// bitwise deterministic without sorting and without floating-point atomics.
// The force field lives only on flagged tiles ([slot][3][512] float32); the lattice
// step adds it where tile_slot >= 0.
//
// Interpolation (Eq. (33)) first evaluates the fluid velocity on the flagged tiles
// (one workgroup per tile, pull + moments), then gathers 64 weighted values per node
// in a fixed order; cells outside flagged tiles (a node that moved since the spread)
// are evaluated on the fly.
#include "lbm_internal.h"

namespace lbmib {

constexpr int REC = 20;  // floats per node record: base xyz, channel, w[3][4], F[3], pad

// Stencil base floor(X) - 1 and the four weights phi(base + k - X), k = 0..3.
// Cosine kernel (Eq. (36)) with t = X - floor(X): phi(-1-t) = (1 - sin(pi t/2))/4,
// phi(-t) = (1 + cos(pi t/2))/4, phi(1-t) = (1 + sin(pi t/2))/4, phi(2-t) = (1 - cos(pi t/2))/4.
// Peskin 4-point kernel with q = sqrt(1 + 4t - 4t^2): (3-2t-q)/8, (3-2t+q)/8, (1+2t+q)/8,
// (1+2t-q)/8.
__device__ __forceinline__ int64_t ib_weights(int kernel, double X, float w[4]) {
    const double fl = floor(X);
    const float t = (float)(X - fl);
    if (kernel == IB_PHI_COS4) {
        float s, c;
        sincospif(0.5f * t, &s, &c);
        w[0] = 0.25f * (1.0f - s);
        w[1] = 0.25f * (1.0f + c);
        w[2] = 0.25f * (1.0f + s);
        w[3] = 0.25f * (1.0f - c);
    } else {
        const float q = sqrtf(fmaxf(1.0f + 4.0f * t - 4.0f * t * t, 0.0f));
        w[0] = 0.125f * (3.0f - 2.0f * t - q);
        w[1] = 0.125f * (3.0f - 2.0f * t + q);
        w[2] = 0.125f * (1.0f + 2.0f * t + q);
        w[3] = 0.125f * (1.0f + 2.0f * t - q);
    }
    return (int64_t)fl - 1;
}

__device__ __forceinline__ int wrapi(int64_t a, int n) {
    int64_t r = a % n;
    return (int)(r < 0 ? r + n : r);
}

// Distinct tiles (of TILE cells) of up to 4 cells; returns the count (<= 4).
__device__ __forceinline__ int distinct_tiles(const int cells[4], const bool ok[4], int out[4]) {
    int k = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (!ok[a]) continue;
        const int t = cells[a] >> 3;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen |= (out[j] == t);
        if (!seen) out[k++] = t;
    }
    return k;
}

struct Stencil {
    int x[4], y[4], z[4];
    bool yok[4];
};

// Cells of the 4x4x4 stencil of a node whose (wrapped) base is bx, by, bz.
__device__ __forceinline__ void stencil_cells(const Chan& ch, int bx, int by, int bz, Stencil& s) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int xc = bx + k;
        s.x[k] = xc >= ch.nx ? xc - ch.nx : xc;
        int zc = bz + k;
        s.z[k] = zc >= ch.nz ? zc - ch.nz : zc;
        int yc = by + k;
        if (ch.walls) {
            s.yok[k] = yc >= 0 && yc < ch.ny;
            s.y[k] = yc;
        } else {
            s.yok[k] = true;
            s.y[k] = yc >= ch.ny ? yc - ch.ny : yc;
        }
    }
}

// ---------------------------------------------------------------- bin
// One thread per node, 256 nodes per block.  Tile counts are first aggregated per block in
// an LDS hash (tile id -> count), then added to the global counter with one atomic per
// (block, tile); a node's rank inside a tile's list is the block's base (kept per hash entry
// in `blkbase`) plus its rank inside the block (kept packed in `rank`).  With nodes numbered
// along the surface a block touches a few tiles, so global atomics drop from one per
// (node, tile) to a few per block.
constexpr int MAXT = 27;   // most tiles a 4x4x4 stencil can touch

__device__ __forceinline__ int chan_of_tile(const Chan* chan, int nch, int64_t T) {
    int lo = 0, hi = nch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chan[mid].tile_off <= T) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void append_flagged(const IbArgs& a, int64_t T) {
    const int slot = atomicAdd(&a.set.hdr->nflag, 1);
    a.set.flag_list[slot] = (int32_t)T;
    a.set.flag_ch[slot] = chan_of_tile(a.chan, a.nch, T);
}

// Tiles touched by the stencil of a node, in a fixed order (z outer, x inner).
template <class F>
__device__ __forceinline__ void for_tiles(const Chan& ch, int bx, int by, int bz, F f) {
    Stencil s;
    stencil_cells(ch, bx, by, bz, s);
    bool all[4] = {true, true, true, true};
    int tx[4], ty[4], tz[4];
    const int nxt = distinct_tiles(s.x, all, tx);
    const int nyt = distinct_tiles(s.y, s.yok, ty);
    const int nzt = distinct_tiles(s.z, all, tz);
    int q = 0;
    for (int k = 0; k < nzt; ++k)
        for (int j = 0; j < nyt; ++j)
            for (int i = 0; i < nxt; ++i)
                f(q++, ch.tile_off + tx[i] + (int64_t)ch.tnx * (ty[j] + (int64_t)ch.tny * tz[k]));
}

// Distinct tiles of `cnt` (4 or 5) consecutive cells from `start` along an axis of `dim` cells
// (periodic, or cut at the walls when `bounded`): at most three.
__device__ __forceinline__ int axis_tiles(int start, int cnt, int dim, bool bounded, int out[3]) {
    int k = 0;
    for (int a = 0; a < cnt; ++a) {
        int c = start + a;
        if (bounded) {
            if (c < 0 || c >= dim) continue;
        } else {
            c = c >= dim ? c - dim : c;
        }
        const int t = c >> 3;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen |= (out[j] == t);
        if (!seen && k < 3) out[k++] = t;
    }
    return k;
}

// Tiles reachable by a node binned with a margin: the stencils of every base from lo to hi
// (per axis, unwrapped), i.e. the cells lo - 1 .. hi + 2.  Same order as for_tiles.
template <class F>
__device__ __forceinline__ void for_tiles_margin(const Chan& ch, const int4 lo, const int4 hi, F f) {
    int tx[3], ty[3], tz[3];
    const int nxt = axis_tiles(wrapi((int64_t)lo.x - 1, ch.nx), hi.x - lo.x + 4, ch.nx, false, tx);
    const int nyt = ch.walls ? axis_tiles(lo.y - 1, hi.y - lo.y + 4, ch.ny, true, ty)
                             : axis_tiles(wrapi((int64_t)lo.y - 1, ch.ny), hi.y - lo.y + 4, ch.ny, false, ty);
    const int nzt = axis_tiles(wrapi((int64_t)lo.z - 1, ch.nz), hi.z - lo.z + 4, ch.nz, false, tz);
    int q = 0;
    for (int k = 0; k < nzt; ++k)
        for (int j = 0; j < nyt; ++j)
            for (int i = 0; i < nxt; ++i)
                f(q++, ch.tile_off + tx[i] + (int64_t)ch.tnx * (ty[j] + (int64_t)ch.tny * tz[k]));
}

// floor(X - margin) and floor(X + margin) per axis, the y range clamped like the stencil base
// of a node outside the channel.
__device__ __forceinline__ void margin_range(const Chan& ch, const double* X, int64_t n, int64_t m, double margin,
                                             int4& lo, int4& hi) {
    int l[3], h[3];
    for (int d = 0; d < 3; ++d) {
        const double x = X[d * n + m];
        const bool finite = isfinite(x) && fabs(x) < 1e9;
        int64_t a = finite ? (int64_t)floor(x - margin) : 0, b = finite ? (int64_t)floor(x + margin) : 0;
        if (d == 1 && ch.walls) {
            a = a < -3 ? -3 : (a > ch.ny + 1 ? ch.ny + 1 : a);
            b = b < -3 ? -3 : (b > ch.ny + 1 ? ch.ny + 1 : b);
        }
        if (b - a > 1) b = a + 1;  // margin < 1/2 keeps b - a <= 1
        l[d] = (int)a;
        h[d] = (int)b;
    }
    lo = make_int4(l[0], l[1], l[2], 0);
    hi = make_int4(h[0], h[1], h[2], 0);
}

// Axis d of node m's record: the stencil base floor(X) - 1 (x, z wrapped; y clamped for a node
// outside the channel) and the four kernel weights; returns the base and whether the node lies
// outside the channel (or is not finite) along this axis.
__device__ __forceinline__ int record_axis(const IbArgs& a, int64_t m, const Chan& ch, int d, bool& bad) {
    float* r = a.rec + m * REC;
    float w[4];
    const double X = a.X[d * a.n + m];
    const int dim = d == 0 ? ch.nx : (d == 1 ? ch.ny : ch.nz);
    const bool finite = isfinite(X) && fabs(X) < 1e9;
    int64_t base = finite ? ib_weights(a.kernel, X, w) : 0;
    bad = !finite;
    if (!finite) w[0] = w[1] = w[2] = w[3] = 0.0f;
    int b;
    if (d == 1 && ch.walls) {
        // node outside the channel: y outside [-1, ny), or [0, ny-1] with on-site walls
        if (ch.walls == 2 ? (X < 0.0 || X > ch.ny - 1.0) : (base < -2 || base > ch.ny - 2)) bad = true;
        if (base < -4) base = -4;
        if (base > ch.ny) base = ch.ny;
        b = (int)base;
    } else {
        b = wrapi(base, dim);
    }
    r[d] = __int_as_float(b);
    for (int k = 0; k < 4; ++k) r[4 + 4 * d + k] = w[k];
    return b;
}

// The whole record of node m (channel c): the three axes and the channel; sets
// LBM_FLAG_NODE_OUTSIDE for a node outside the channel or not finite.
__device__ __forceinline__ void node_record(const IbArgs& a, int64_t m, int c, const Chan& ch, int b[3]) {
    bool bad = false;
    for (int d = 0; d < 3; ++d) {
        bool bd;
        b[d] = record_axis(a, m, ch, d, bd);
        bad |= bd;
    }
    if (bad) atomicOr(a.flags, LBM_FLAG_NODE_OUTSIDE);
    a.rec[m * REC + 3] = __int_as_float(c);
}

// One block of the binning (256 nodes; `blk` is its index among the bin blocks).  With
// `with_f` it also copies F into the node records and reduces max |F| for the scan; without,
// the membrane-force kernel that runs after it does both (the coupled step).
__device__ __forceinline__ void bin_block(const IbArgs& a, int64_t blk, bool with_f) {
    __shared__ int hkey[HS];
    __shared__ int hcnt[HS];
    __shared__ float wmax[4];
    for (int e = threadIdx.x; e < HS; e += blockDim.x) {
        hkey[e] = -1;
        hcnt[e] = 0;
    }
    __syncthreads();
    const int64_t m = blk * blockDim.x + threadIdx.x;
    float fm = 0.0f;
    if (m < a.n) {
        const int c = a.node_ch[m];
        const Chan& ch = a.chan[c];
        float* r = a.rec + m * REC;
        int b[3];
        node_record(a, m, c, ch, b);
        if (with_f)
            for (int d = 0; d < 3; ++d) {
                const float F = a.F[d * a.n + m];
                r[16 + d] = F;
                fm = fmaxf(fm, fabsf(F));
                if (!isfinite(F)) fm = __uint_as_float(0x7f800000u);
            }
        int32_t* rk = a.rank + m * MAXT;
        auto hash_tile = [&](int q, int64_t T) {
            int h = (int)(((uint32_t)T * 2654435761u) >> (32 - HS_BITS)) & (HS - 1);
            int packed = INT32_MIN;
            for (int probe = 0; probe < 64; ++probe) {
                const int old = atomicCAS(&hkey[h], -1, (int)T);
                if (old == -1 || old == (int)T) {
                    packed = (h << 16) | atomicAdd(&hcnt[h], 1);
                    break;
                }
                h = (h + 1) & (HS - 1);
            }
            if (packed == INT32_MIN) {  // block table full: count this one directly
                const int rr = atomicAdd(&a.set.cnt[T], 1);
                if (rr == 0) append_flagged(a, T);
                packed = -(rr + 1);
            }
            rk[q] = packed;
        };
        if (a.margin > 0.0) {
            int4 lo, hi;
            margin_range(ch, a.X, a.n, m, a.margin, lo, hi);
            a.nbin[2 * m] = lo;
            a.nbin[2 * m + 1] = hi;
            for_tiles_margin(ch, lo, hi, hash_tile);
        } else {
            for_tiles(ch, b[0], b[1], b[2], hash_tile);
        }
    }
    // block maximum of |F| (NaN/Inf bits compare above all finite values)
    uint32_t ub = __float_as_uint(fm);
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(ub, d, 64);
        ub = o > ub ? o : ub;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = __uint_as_float(ub);
    __syncthreads();
    // only the entries in use are read back (by the scatter)
    int32_t* bb = a.blkbase + blk * HS;
    for (int e = threadIdx.x; e < HS; e += blockDim.x) {
        const int T = hkey[e];
        if (T >= 0) {
            const int base = atomicAdd(&a.set.cnt[T], hcnt[e]);
            if (base == 0) append_flagged(a, T);
            bb[e] = base;
        }
    }
    if (with_f && threadIdx.x == 0) {
        uint32_t mx = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            const uint32_t v = __float_as_uint(wmax[k]);
            mx = v > mx ? v : mx;
        }
        a.blkmax[blk] = mx;  // reduced by the scan
    }
}

__global__ void __launch_bounds__(256) k_ib_bin(IbArgs a) { bin_block(a, blockIdx.x, true); }

// ---------------------------------------------------------------- scan (one workgroup)
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// max |F| over the per-workgroup maxima in blkmax and the spread's fixed-point scale from it
// (set.hdr: fmax_bits, nonfinite, scale_exp).  Every thread of one workgroup calls it.
__device__ __forceinline__ int scale_exponent(float fm, int64_t n) {
    // fixed-point scale: |contribution| <= max|F|/8 and at most n contributions per
    // cell, so |sum| < n * 2^e / 8 with max|F| < 2^e; keep sums below 2^62.
    int s = 0;
    if (isfinite(fm) && fm > 0.0f) {
        int e;
        const float m = frexpf(fm, &e);  // fm = m 2^e, 1/2 <= m < 1
        // a force within 2^-16 of the next power of two takes the next exponent: the margin
        // absorbs the float rounding of the weights (each 1/2 at most, up to an ulp)
        if (m > 1.0f - 0x1p-16f) ++e;
        int L = 1;
        while ((1ll << L) < n) ++L;
        // one contribution |w_x w_y w_z F| <= (1 + 2^-20) max|F|/8 < (1 - 2^-17) 2^(e-3)
        // stays below 2^23 - 64 at the spread's per-batch scale 2^(s-8), also once rounded
        // to an integer, so a batch of <= 256 of them sums to less than 2^31 and converts
        // exactly through int32; a sum of <= n of them stays below 2^62; the quantum of a
        // contribution is 2^-26 max|F| or finer (2^-25 in the margin)
        s = 34 - e;
        if (s > 65 - e - L) s = 65 - e - L;
    }
    return s;
}

// max |F| over the per-workgroup maxima in blkmax (float bits; NaN/Inf above every finite
// value), reduced by the calling workgroup; every thread gets it.
__device__ __forceinline__ uint32_t force_max_bits(const IbArgs& a) {
    __shared__ uint32_t fmx[16];
    __shared__ uint32_t all;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbk = (int)a.blkmax_n;
    uint32_t mx = 0;
    for (int k = tid; k < nbk; k += blockDim.x) {
        const uint32_t v = a.blkmax[k];
        mx = v > mx ? v : mx;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    if (lane == 0) fmx[wave] = mx;
    __syncthreads();
    if (tid == 0) {
        uint32_t mxall = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mxall = fmx[w] > mxall ? fmx[w] : mxall;
        all = mxall;
    }
    __syncthreads();
    return all;
}

// max |F| and the spread's fixed-point scale from it into set.hdr (fmax_bits, nonfinite,
// scale_exp).  Every thread of one workgroup calls it.
__device__ __forceinline__ void spread_scale(const IbArgs& a) {
    const uint32_t mxall = force_max_bits(a);
    if (threadIdx.x == 0) {
        const float fm = __uint_as_float(mxall);
        a.set.hdr->fmax_bits = mxall;
        if (!isfinite(fm)) {
            a.set.hdr->nonfinite = 1;
            atomicOr(a.flags, LBM_FLAG_FORCE_NONFINITE);
        }
        a.set.hdr->scale_exp = scale_exponent(fm, a.n);
    }
}

// One workgroup: list offsets, work items and partial-block offsets of the flagged tiles;
// with_scale: also the spread's scale (else the scatter's first workgroup computes it, once
// the membrane forces are in).
__device__ __forceinline__ void scan_block(const IbArgs& a, bool with_scale) {
    __shared__ int wsum[3][16];
    __shared__ int carry[3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // clear the tile set used by the spread before last
    const int nfo = a.other.hdr->nflag;
    for (int k = tid; k < nfo; k += blockDim.x) {
        const int T = a.other.flag_list[k];
        a.other.cnt[T] = 0;
        a.other.tile_slot[T] = -1;
    }
    const int nf = a.set.hdr->nflag;
    if (tid < 3) carry[tid] = 0;
    __syncthreads();  // every thread has read the other set's count before it is reset below
    // three exclusive prefixes over the flagged tiles: list offsets (node count), spread
    // work items (chunks of a.chunk nodes) and the partial blocks of split tiles
    for (int base = 0; base < nf; base += blockDim.x) {
        const int k = base + tid;
        const int v = k < nf ? a.set.cnt[a.set.flag_list[k]] : 0;
        const int ck = a.chunk;
        const int nch = k < nf ? (v > ck ? (v + ck - 1) / ck : 1) : 0;
        const int val[3] = {v, nch, nch > 1 ? nch : 0};
        int incl[3], excl[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            incl[j] = wave_incl_scan(val[j]);
            if (lane == 63) wsum[j][wave] = incl[j];
        }
        __syncthreads();
        if (wave == 0) {
            const int nw = blockDim.x >> 6;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                int x = lane < nw ? wsum[j][lane] : 0;
                x = wave_incl_scan(x);
                if (lane < nw) wsum[j][lane] = x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 3; ++j) excl[j] = carry[j] + (wave ? wsum[j][wave - 1] : 0) + incl[j] - val[j];
        if (k < nf) {
            a.set.slot_off[k] = excl[0];
            a.set.tile_slot[a.set.flag_list[k]] = k;
            a.set.chunk_off[k] = excl[1];
            a.set.big[k] = (val[2] && (int64_t)excl[2] + val[2] <= a.part_cap) ? excl[2] : -1;
            for (int j = 0; j < nch && (int64_t)excl[1] + j < a.max_items; ++j) a.item_slot[excl[1] + j] = k;
        }
        __syncthreads();
        if (tid == blockDim.x - 1)
#pragma unroll
            for (int j = 0; j < 3; ++j) carry[j] = excl[j] + val[j];
        __syncthreads();
    }
    if (with_scale) spread_scale(a);
    if (tid == 0) {
        const int total = carry[0];
        a.set.slot_off[nf] = total;
        a.set.chunk_off[nf] = carry[1];
        a.set.hdr->nchunk = (int64_t)carry[1] < a.max_items ? carry[1] : (int)a.max_items;
        a.other.hdr->nchunk = 0;
        a.other.hdr->nflag = 0;
        a.other.hdr->fmax_bits = 0;
        a.other.hdr->nonfinite = 0;
        a.other.hdr->scale_exp = 0;
        if (total > a.list_cap) atomicOr(a.flags, LBM_FLAG_LIST_OVERFLOW);
    }
}

__global__ void __launch_bounds__(1024) k_ib_scan(IbArgs a) { scan_block(a, true); }

// ---------------------------------------------------------------- scatter (no atomics)
__global__ void __launch_bounds__(256) k_ib_scatter(IbArgs a) {
    if (a.scale_in_scatter && blockIdx.x == 0) spread_scale(a);
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n) return;
    const float* r = a.rec + m * REC;
    const Chan& ch = a.chan[__float_as_int(r[3])];
    const int32_t* rk = a.rank + m * MAXT;
    const int32_t* bb = a.blkbase + (m >> 8) * HS;
    auto place = [&](int q, int64_t T) {
        const int packed = rk[q];
        const int rr = packed >= 0 ? bb[packed >> 16] + (packed & 0xffff) : -packed - 1;
        const int slot = a.set.tile_slot[T];
        const int64_t pos = (int64_t)a.set.slot_off[slot] + rr;
        if (pos < a.list_cap) a.list[pos] = (int32_t)m;
    };
    if (a.margin > 0.0)
        for_tiles_margin(ch, a.nbin[2 * m], a.nbin[2 * m + 1], place);
    else
        for_tiles(ch, __float_as_int(r[0]), __float_as_int(r[1]), __float_as_int(r[2]), place);
}

// ---------------------------------------------------------------- spread (LDS, fixed point)
// Work item = one chunk of up to a.chunk nodes of a flagged 8x8x8 tile's node list.  The
// chunk's node records are staged in LDS; then each wavefront takes one node at a time with
// lane = stencil point (x = lane & 3, y = (lane >> 2) & 3, z = lane >> 4): the lanes whose
// cell lies in the tile (and not inside a wall) add w_x w_y w_z F to a 64-bit fixed-point
// LDS accumulator of the tile's 512 cells.  A tile of one chunk writes its force block
// directly; each chunk of a longer list stores its fixed-point partial block, and a second
// kernel adds the tile's blocks and writes the force block.  Integer sums are exact, so the
// result does not depend on the order in which nodes were listed or chunks ran.
constexpr int SP_THREADS = 512;   // 8 wavefronts per work item (four work items per CU)
constexpr int SP_BATCH = 256;     // node records staged at a time (a chunk is spread in batches)

__device__ __forceinline__ unsigned fixed_round(float c, float scale) {
    // round-to-nearest-even of c * scale (a power of two: the product is exact) for
    // |c * scale| < 2^23 - 64, as a two's-complement 32-bit word
    return (unsigned)(int)__builtin_rintf(c * scale);
}

// Contributions are summed per staged batch in 32-bit LDS words (cheaper atomics than 64-bit
// ones), at 2^-8 of the tile accumulator's scale: each rounds to less than 2^23 - 64 there and
// a batch adds at most SP_BATCH of them to a cell, so a batch sum stays below 2^31 and is exact.
// After each batch the words are added, scaled by 2^8, to the tile's 64-bit accumulator.
constexpr int SP_BATCH_SHIFT = 8;
static_assert(SP_BATCH <= (1 << SP_BATCH_SHIFT), "a batch sum must stay below 2^31");

// The spread's work items first, first + stride, ... (one workgroup of SP_THREADS threads).
__device__ __forceinline__ void spread_items(const IbArgs& a, int64_t first, int64_t stride) {
    __shared__ unsigned long long acc[3 * TILE_CELLS];
    __shared__ unsigned acc32[3 * TILE_CELLS];
    __shared__ int4 base[SP_BATCH];         // stencil base x, y, z of each staged node
    __shared__ float4 wrec[SP_BATCH][4];    // w_x[4], w_y[4], w_z[4], (F, pad)
    const int nwork = a.set.hdr->nchunk;
    int sexp;
    bool nonfinite;
    if (a.scale_local) {
        // between binnings no launch before the spread reduces the force maximum: every work
        // item reduces it itself, and the first one records it for the later readers
        const uint32_t mb = force_max_bits(a);
        const float fm = __uint_as_float(mb);
        nonfinite = !isfinite(fm);
        sexp = scale_exponent(fm, a.n);
        if (first == 0 && threadIdx.x == 0) {
            a.set.hdr->fmax_bits = mb;
            a.set.hdr->nonfinite = nonfinite ? 1 : 0;
            a.set.hdr->scale_exp = sexp;
            if (nonfinite) atomicOr(a.flags, LBM_FLAG_FORCE_NONFINITE);
        }
    } else {
        sexp = a.set.hdr->scale_exp;
        nonfinite = a.set.hdr->nonfinite != 0;
    }
    const float scale = ldexpf(1.0f, sexp - SP_BATCH_SHIFT);
    const double inv = ldexp(1.0, -sexp);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ix = lane & 3, iy = (lane >> 2) & 3, iz = lane >> 4;
    for (int64_t wi = first; wi < nwork; wi += stride) {
        const int slot = a.item_slot[wi];
        const int c = wi - a.set.chunk_off[slot];
        const int nch = a.set.chunk_off[slot + 1] - a.set.chunk_off[slot];
        const int bigid = a.set.big[slot];
        const bool split = nch > 1 && bigid >= 0;
        if (nch > 1 && bigid < 0 && c != 0) continue;  // no accumulator left: chunk 0 takes the list
        int64_t beg = a.set.slot_off[slot], end = a.set.slot_off[slot + 1];
        if (split) {
            beg += (int64_t)c * a.chunk;
            if (end > beg + a.chunk) end = beg + a.chunk;
        }
        if (end > a.list_cap) end = a.list_cap;
        for (int k = tid; k < 3 * TILE_CELLS; k += SP_THREADS) {
            acc[k] = 0ull;
            acc32[k] = 0u;
        }
        const int T = a.set.flag_list[slot];
        // the channel's fields in registers: read through the descriptor, the node loop below
        // would load them again from memory after every LDS atomic
        const Chan& ch = a.chan[a.set.flag_ch[slot]];
        const int cnx = ch.nx, cny = ch.ny, cnz = ch.nz;
        const int t = (int)(T - ch.tile_off);
        const int tx0 = (t % ch.tnx) * TILE;
        const int ty0 = ((t / ch.tnx) % ch.tny) * TILE;
        const int tz0 = (t / (ch.tnx * ch.tny)) * TILE;
        const bool wrap_y = !ch.walls;
        for (int64_t b0 = beg; b0 < end; b0 += SP_BATCH) {
            const int nb = (int)(end - b0 < SP_BATCH ? end - b0 : SP_BATCH);
            __syncthreads();  // the previous batch is consumed (and acc is cleared)
            for (int k = tid; k < nb; k += SP_THREADS) {
                const int64_t m = a.list[b0 + k];
                const float4* r = (const float4*)(a.rec + m * REC);
                const float4 r0 = r[0];
                base[k] = make_int4(__float_as_int(r0.x), __float_as_int(r0.y), __float_as_int(r0.z), 0);
                wrec[k][0] = r[1];
                wrec[k][1] = r[2];
                wrec[k][2] = r[3];
                wrec[k][3] = r[4];
            }
            __syncthreads();
            for (int q = wave; q < nb; q += SP_THREADS / 64) {
                const int4 bq = base[q];
                int cx = bq.x + ix, cy = bq.y + iy, cz = bq.z + iz;
                if (cx >= cnx) cx -= cnx;
                if (cz >= cnz) cz -= cnz;
                bool ok = true;
                if (wrap_y) {
                    if (cy >= cny) cy -= cny;
                } else {
                    ok = cy >= 0 && cy < cny;
                }
                const int lx = cx - tx0, ly = cy - ty0, lz = cz - tz0;
                if (ok && (unsigned)lx < (unsigned)TILE && (unsigned)ly < (unsigned)TILE && (unsigned)lz < (unsigned)TILE) {
                    const float* w = (const float*)wrec[q];
                    const float ww = w[ix] * (w[4 + iy] * w[8 + iz]);
                    const int loc = (lz << 6) | (ly << 3) | lx;
                    atomicAdd(&acc32[loc], fixed_round(ww * w[12], scale));
                    atomicAdd(&acc32[TILE_CELLS + loc], fixed_round(ww * w[13], scale));
                    atomicAdd(&acc32[2 * TILE_CELLS + loc], fixed_round(ww * w[14], scale));
                }
            }
            __syncthreads();
            for (int k = tid; k < 3 * TILE_CELLS; k += SP_THREADS) {
                acc[k] += (unsigned long long)((long long)(int)acc32[k] * (1ll << SP_BATCH_SHIFT));
                acc32[k] = 0u;
            }
        }
        __syncthreads();
        float* out = a.force + (int64_t)slot * (3 * TILE_CELLS);
        if (!split) {
            for (int k = tid; k < 3 * TILE_CELLS; k += SP_THREADS)
                out[k] = nonfinite ? __builtin_nanf("") : (float)((double)(long long)acc[k] * inv);
        } else {
            // this chunk's partial block; k_ib_merge adds the tile's blocks
            unsigned long long* pb = a.part + ((int64_t)bigid + c) * (3 * TILE_CELLS);
            for (int k = tid; k < 3 * TILE_CELLS; k += SP_THREADS) pb[k] = acc[k];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SP_THREADS) k_ib_spread(IbArgs a) { spread_items(a, blockIdx.x, gridDim.x); }

// The spread's work items (workgroups [0, gs)) beside the lattice update of every cell with
// the body force alone (the rest, SP_THREADS/64 segments of 64 cells each), which does not
// depend on the spread; the flagged tiles' cells are updated again afterwards with their
// force (k_step_tiles).  Same helpers and roundings as the fused step.
template <class St, bool NT>
__global__ void __launch_bounds__(SP_THREADS) k_spread_far(IbArgs a, LatArgs la, int64_t gs) {
    using T = typename St::T;
    if ((int64_t)blockIdx.x < gs) {
        spread_items(a, blockIdx.x, gs);
        return;
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t sw = ((int64_t)blockIdx.x - gs) * (SP_THREADS / 64) + wave;
    if (sw >= la.nseg) return;
    const int64_t seg = la.reverse ? la.nseg - 1 - sw : sw;
    const Chan& ch = la.chan[la.seg_ch[seg]];
    const int64_t n64 = (seg - ch.seg_off) * 64 + lane;
    if (n64 >= ch.ncell) return;
    const int32_t n = (int32_t)n64;
    int x, y, z;
    cell_xyz(ch, (uint32_t)n, x, y, z);
    const T* src = (const T*)la.src + ch.pop_off;
    T* dst = (T*)la.dst + ch.pop_off;
    float g[Q];
    pull<St>(src, ch, ch.ncell, n, x, y, z, g);
    if (St::onsite && onsite_row(ch, y)) onsite_wall(ch, y, g, ch.body[0], ch.body[1], ch.body[2]);
    float drho, jx, jy, jz;
    moments(g, drho, jx, jy, jz);
    const CellState cs = cell_state(drho, jx, jy, jz, ch.body[0], ch.body[1], ch.body[2]);
    const float om = ch.omega, guo = ch.guo;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float gn = bgk_c(i, g[i], cs, om, guo);
        if (NT)
            St::st_nt(dst + pidx(i, n), gn);
        else
            St::st(dst + pidx(i, n), gn);
    }
}

template <class St>
static void launch_spread_far_typed(lbm_ctx* c, const IbArgs& a, const LatArgs& la, int64_t gs, int64_t gl) {
    const dim3 grid((unsigned)(gs + gl)), block(SP_THREADS);
    if (c->launch.nontemporal)
        k_spread_far<St, true><<<grid, block, 0, c->stream>>>(a, la, gs);
    else
        k_spread_far<St, false><<<grid, block, 0, c->stream>>>(a, la, gs);
}

hipError_t launch_spread_far(lbm_ctx* c, const IbArgs& a, const LatArgs& la) {
    int64_t gs = c->max_items < c->ib_grid ? c->max_items : c->ib_grid;
    if (gs < 1) gs = 1;
    const int64_t gl = (la.nseg + SP_THREADS / 64 - 1) / (SP_THREADS / 64);
    with_storage(c, [&](auto st) { launch_spread_far_typed<decltype(st)>(c, a, la, gs, gl); });
    return hipGetLastError();
}

// Force blocks of split tiles: the sum of their chunks' partial blocks (chunk order).
constexpr int MG_THREADS = 512;
__global__ void __launch_bounds__(MG_THREADS) k_ib_merge(IbArgs a) {
    const int nf = a.set.hdr->nflag;
    const bool nonfinite = a.set.hdr->nonfinite != 0;
    const double inv = ldexp(1.0, -a.set.hdr->scale_exp);
    for (int slot = blockIdx.x; slot < nf; slot += gridDim.x) {
        const int bigid = a.set.big[slot];
        if (bigid < 0) continue;
        const int nch = a.set.chunk_off[slot + 1] - a.set.chunk_off[slot];
        const unsigned long long* pb = a.part + (int64_t)bigid * (3 * TILE_CELLS);
        float* out = a.force + (int64_t)slot * (3 * TILE_CELLS);
        for (int k = threadIdx.x; k < 3 * TILE_CELLS; k += MG_THREADS) {
            unsigned long long v = 0ull;
            for (int j0 = 0; j0 < nch; j0 += 8) {
                unsigned long long t[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] = j0 + u < nch ? pb[(int64_t)(j0 + u) * (3 * TILE_CELLS) + k] : 0ull;
#pragma unroll
                for (int u = 0; u < 8; ++u) v += t[u];
            }
            out[k] = nonfinite ? __builtin_nanf("") : (float)((double)(long long)v * inv);
        }
    }
}

hipError_t launch_ib_spread(lbm_ctx* c, const IbArgs& a) {
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    if (a.n > 0) k_ib_bin<<<dim3(nb), dim3(256), 0, c->stream>>>(a);
    return launch_ib_spread_binned(c, a);
}

// The spread after the binning: scan, scatter, fixed-point spread, merge.
hipError_t launch_ib_spread_binned(lbm_ctx* c, const IbArgs& a) {
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    k_ib_scan<<<dim3(1), dim3(1024), 0, c->stream>>>(a);
    if (a.n > 0) k_ib_scatter<<<dim3(nb), dim3(256), 0, c->stream>>>(a);
    return launch_ib_spread_items(c, a);
}

// Fixed-point spread of the listed nodes and the merge of split tiles.
hipError_t launch_ib_spread_items(lbm_ctx* c, const IbArgs& a) {
    // the number of work items is only known on the device: a grid of a few workgroups per
    // CU walks them (launching one workgroup per possible item costs more in empty waves
    // than the work itself)
    int64_t g = c->max_items < c->ib_grid ? c->max_items : c->ib_grid;
    if (g < 1) g = 1;
    k_ib_spread<<<dim3((unsigned)g), dim3(SP_THREADS), 0, c->stream>>>(a);
    const int64_t gm = c->max_slots < c->ib_grid ? c->max_slots : c->ib_grid;
    k_ib_merge<<<dim3((unsigned)(gm < 1 ? 1 : gm)), dim3(MG_THREADS), 0, c->stream>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- interpolation
// Fluid velocity of the current state, v = (j + (F_body + g)/2)/rho (Eq. (18) and the
// shift under Eq. (19)), on every cell of every flagged tile.
template <class St>
__global__ void __launch_bounds__(512) k_ib_vel(IbArgs a) {
    using T = typename St::T;
    const int nf = a.set.hdr->nflag;
    constexpr int PART = TILE_CELLS / TILE_PARTS;  // cells of a tile per workgroup
    const int part = (int)(blockIdx.x % TILE_PARTS);
    for (int slot = blockIdx.x / TILE_PARTS; slot < nf; slot += gridDim.x / TILE_PARTS) {
        const int T_ = a.set.flag_list[slot];
        const Chan& ch = a.chan[a.set.flag_ch[slot]];
        const int t = (int)(T_ - ch.tile_off);
        const int ox = (t % ch.tnx) * TILE, oy = ((t / ch.tnx) % ch.tny) * TILE, oz = (t / (ch.tnx * ch.tny)) * TILE;
        const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS);
        float4* vb = (float4*)(a.vel + (int64_t)slot * (4 * TILE_CELLS));
        for (int l = part * PART + threadIdx.x; l < (part + 1) * PART; l += blockDim.x) {
            const int x = ox + (l & 7), y = oy + ((l >> 3) & 7), z = oz + (l >> 6);
            if (x >= ch.nx || y >= ch.ny || z >= ch.nz) continue;
            const int32_t n = x + ch.nx * (y + ch.ny * z);
            float g[Q];
            pull<St>((const T*)a.pop + ch.pop_off, ch, ch.ncell, n, x, y, z, g);
            const float Fx = ch.body[0] + fb[l], Fy = ch.body[1] + fb[TILE_CELLS + l],
                        Fz = ch.body[2] + fb[2 * TILE_CELLS + l];
            if (St::onsite && onsite_row(ch, y)) onsite_wall(ch, y, g, Fx, Fy, Fz);
            float drho, jx, jy, jz;
            moments(g, drho, jx, jy, jz);
            const float ir = 1.0f / (1.0f + drho);
            vb[l] = make_float4((jx + 0.5f * Fx) * ir, (jy + 0.5f * Fy) * ir, (jz + 0.5f * Fz) * ir, 0.0f);
        }
    }
}

// U_m = sum over the stencil of v(x) phi phi phi, rows inside a wall taking the wall
// velocity; optionally X_out = X + U.  GL lanes per node (4 or 2): lane l takes the stencil
// rows q = l, l + GL, ... (y = base_y + q % 4, z = base_z + q / 4), each with its four x
// cells; the GL partial sums are combined by a fixed butterfly, so the result does not
// depend on scheduling.  Few nodes (one wave round or so) gain from more lanes per node,
// many nodes from more independent loads per lane (the launch picks GL by the node count).
template <class St, int GL>
__global__ void __launch_bounds__(256) k_ib_gather(IbArgs a) {
    static_assert(GL == 2 || GL == 4 || GL == 8 || GL == 16, "lanes per node");
    constexpr int GR = 16 / GL;  // stencil rows per lane
    using T = typename St::T;
    // consecutive node blocks on the same XCD: neighbouring nodes share tiles in one L2
    const int64_t G = gridDim.x, bx = blockIdx.x, per = G >> 3, rem = G & 7, xcd = bx & 7;
    const int64_t L = xcd * per + (xcd < rem ? xcd : rem) + (bx >> 3);
    const int64_t m = (L * blockDim.x + threadIdx.x) / GL;
    const int sl = threadIdx.x & (GL - 1);
    float U[3] = {0.f, 0.f, 0.f};
    double X[3] = {0.0, 0.0, 0.0};
    const bool valid = m < a.n;
    if (valid) {
        float w[3][4];
        int b[3];
        int c;
        if (a.use_rec) {
            // positions unchanged since the spread: its node record holds base and weights
            const float4* r = (const float4*)(a.rec + m * REC);
            const float4 r0 = r[0], rx = r[1], ry = r[2], rz = r[3];
            b[0] = __float_as_int(r0.x);
            b[1] = __float_as_int(r0.y);
            b[2] = __float_as_int(r0.z);
            c = __float_as_int(r0.w);
            w[0][0] = rx.x; w[0][1] = rx.y; w[0][2] = rx.z; w[0][3] = rx.w;
            w[1][0] = ry.x; w[1][1] = ry.y; w[1][2] = ry.z; w[1][3] = ry.w;
            w[2][0] = rz.x; w[2][1] = rz.y; w[2][2] = rz.z; w[2][3] = rz.w;
            if (a.Xout)
                for (int d = 0; d < 3; ++d) X[d] = a.X[d * a.n + m];
        } else {
            c = a.node_ch[m];
            const Chan& ch = a.chan[c];
            for (int d = 0; d < 3; ++d) {
                X[d] = a.X[d * a.n + m];
                const int dim = d == 0 ? ch.nx : (d == 1 ? ch.ny : ch.nz);
                const bool finite = isfinite(X[d]) && fabs(X[d]) < 1e9;
                int64_t base = finite ? ib_weights(a.kernel, X[d], w[d]) : 0;
                if (!finite) w[d][0] = w[d][1] = w[d][2] = w[d][3] = 0.0f;
                if (d == 1 && ch.walls) {
                    if (base < -4) base = -4;
                    if (base > ch.ny) base = ch.ny;
                    b[d] = (int)base;
                } else {
                    b[d] = wrapi(base, dim);
                }
            }
        }
        const Chan& ch = a.chan[c];
#pragma unroll
        for (int rr = 0; rr < GR; ++rr) {
        const int q = sl + GL * rr, bq = q & 3, cq = q >> 2;
        // this stencil row (y index bq, z index cq), its weights selected without dynamic indexing
        const float wy = bq == 0 ? w[1][0] : (bq == 1 ? w[1][1] : (bq == 2 ? w[1][2] : w[1][3]));
        const float wz = cq == 0 ? w[2][0] : (cq == 1 ? w[2][1] : (cq == 2 ? w[2][2] : w[2][3]));
        const float wyz = wy * wz;
        int y = b[1] + bq;
        bool yok = true;
        if (ch.walls) yok = y >= 0 && y < ch.ny;
        else if (y >= ch.ny) y -= ch.ny;
        int z = b[2] + cq;
        if (z >= ch.nz) z -= ch.nz;
        // the row's four x cells lie in at most two tiles (the first and the last cell's; a
        // middle cell in neither happens only when nx < 8): two slot lookups, not four
        int xs4[4], sl4[4];
        if (yok) {
#pragma unroll
            for (int ax = 0; ax < 4; ++ax) {
                int x = b[0] + ax;
                if (x >= ch.nx) x -= ch.nx;
                xs4[ax] = x;
            }
            const int sa = a.set.tile_slot[tile_of(ch, xs4[0], y, z)];
            const int sb = a.set.tile_slot[tile_of(ch, xs4[3], y, z)];
#pragma unroll
            for (int ax = 0; ax < 4; ++ax) {
                const int tx = xs4[ax] >> 3;
                sl4[ax] = tx == (xs4[0] >> 3) ? sa
                                              : (tx == (xs4[3] >> 3) ? sb : a.set.tile_slot[tile_of(ch, xs4[ax], y, z)]);
            }
        }
#pragma unroll
        for (int ax = 0; ax < 4; ++ax) {
            const float ww = w[0][ax] * wyz;
            float v0, v1, v2;
            if (!yok) {
                const float* uw = y < 0 ? ch.uw_lo : ch.uw_hi;
                v0 = uw[0]; v1 = uw[1]; v2 = uw[2];
            } else {
                const int x = xs4[ax];
                const int slot = sl4[ax];
                if (slot >= 0) {
                    const float4 vb = ((const float4*)(a.vel + (int64_t)slot * (4 * TILE_CELLS)))[tile_local(x, y, z)];
                    v0 = vb.x; v1 = vb.y; v2 = vb.z;
                } else {  // not under any spread stencil: no IB force here
                    const int32_t n = x + ch.nx * (y + ch.ny * z);
                    float g[Q];
                    pull<St>((const T*)a.pop + ch.pop_off, ch, ch.ncell, n, x, y, z, g);
                    if (St::onsite && onsite_row(ch, y)) onsite_wall(ch, y, g, ch.body[0], ch.body[1], ch.body[2]);
                    float drho, jx, jy, jz;
                    moments(g, drho, jx, jy, jz);
                    const float ir = 1.0f / (1.0f + drho);
                    v0 = (jx + 0.5f * ch.body[0]) * ir;
                    v1 = (jy + 0.5f * ch.body[1]) * ir;
                    v2 = (jz + 0.5f * ch.body[2]) * ir;
                }
            }
            U[0] += ww * v0;
            U[1] += ww * v1;
            U[2] += ww * v2;
        }
        }
    }
#pragma unroll
    for (int d = 1; d < GL; d <<= 1) {
        U[0] += __shfl_xor(U[0], d, 64);
        U[1] += __shfl_xor(U[1], d, 64);
        U[2] += __shfl_xor(U[2], d, 64);
    }
    if (valid && sl == 0) {
        for (int d = 0; d < 3; ++d) {
            if (a.U) a.U[d * a.n + m] = U[d];
            if (a.Xout) a.Xout[d * a.n + m] = X[d] + (double)U[d];
        }
    }
}

template <class St>
static void launch_interp_typed(lbm_ctx* c, const IbArgs& a) {
    int64_t g = c->max_slots < c->ib_grid / 2 ? c->max_slots : c->ib_grid / 2;
    if (g < 1) g = 1;
    k_ib_vel<St><<<dim3((unsigned)(g * TILE_PARTS)), dim3(TILE_CELLS / TILE_PARTS), 0, c->stream>>>(a);
    // lanes per node by the node count (measured on 20k, 41k and 0.5 M nodes): 16 while even
    // that is under one round of waves (32768 nodes), 4 up to about one round at 4 lanes
    // (131072 nodes), 2 beyond
    if (a.n > 131072)
        k_ib_gather<St, 2><<<dim3((unsigned)((2 * a.n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
    else if (a.n > 32768)
        k_ib_gather<St, 4><<<dim3((unsigned)((4 * a.n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
    else if (a.n > 0)
        k_ib_gather<St, 16><<<dim3((unsigned)((16 * a.n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
}

hipError_t launch_ib_interp(lbm_ctx* c, const IbArgs& a) {
    with_storage(c, [&](auto st) { launch_interp_typed<decltype(st)>(c, a); });
    return hipGetLastError();
}

__global__ void k_ib_advance(int64_t n3, double* X, const float* U) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n3) X[k] += (double)U[k];
}

hipError_t launch_ib_advance(hipStream_t s, int64_t n, double* X, const float* U) {
    if (n <= 0) return hipSuccess;
    k_ib_advance<<<dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s>>>(3 * n, X, U);
    return hipGetLastError();
}

// ---------------------------------------------------------------- membrane forces
__device__ __forceinline__ void ld3(const double* X, int64_t n, int64_t i, double o[3]) {
    o[0] = X[i];
    o[1] = X[n + i];
    o[2] = X[2 * n + i];
}
__device__ __forceinline__ void sub(const double a[3], const double b[3], double o[3]) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
__device__ __forceinline__ void crs(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dt3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Signed dihedral angle of hinge (x0, x1, x2, x3) about the shared edge e = x2 - x1,
// between the normals nA = (x1-x0) x (x2-x0) and nB = (x2-x3) x (x1-x3), and its gradient
// with respect to the four vertices:
//   d/dx0 = -|e| nA/|nA|^2,  d/dx3 = -|e| nB/|nB|^2,
//   d/dx1 = -((x0-x2).e/|e|) nA/|nA|^2 - ((x3-x2).e/|e|) nB/|nB|^2,
//   d/dx2 =  ((x0-x1).e/|e|) nA/|nA|^2 + ((x3-x1).e/|e|) nB/|nB|^2.
// Returns cos(theta) and sin(theta); the energy only needs
// sin(theta - theta0) = sin(theta) cos(theta0) - cos(theta) sin(theta0).
__device__ void hinge(const double x[4][3], double grad[4][3], bool want_grad, double& cth, double& sth) {
    double a[3], b[3], nA[3], nB[3], e[3], cr[3];
    sub(x[1], x[0], a); sub(x[2], x[0], b); crs(a, b, nA);
    sub(x[2], x[3], a); sub(x[1], x[3], b); crs(a, b, nB);
    sub(x[2], x[1], e);
    const double AA = dt3(nA, nA), BB = dt3(nB, nB), L = sqrt(dt3(e, e));
    const double iab = 1.0 / sqrt(AA * BB);
    // one reciprocal each instead of a division per use (FP64 division is a long sequence)
    const double iL = 1.0 / L;
    crs(nA, nB, cr);
    cth = dt3(nA, nB) * iab;
    sth = dt3(cr, e) * iab * iL;
    if (want_grad) {
        double t0[3], t3[3];
        sub(x[0], x[2], t0); sub(x[3], x[2], t3);
        const double c1A = -dt3(t0, e) * iL, c1B = -dt3(t3, e) * iL;
        sub(x[0], x[1], t0); sub(x[3], x[1], t3);
        const double c2A = dt3(t0, e) * iL, c2B = dt3(t3, e) * iL;
        const double iA = 1.0 / AA, iB = 1.0 / BB;
        for (int d = 0; d < 3; ++d) {
            const double qA = nA[d] * iA, qB = nB[d] * iB;
            grad[0][d] = -L * qA;
            grad[3][d] = -L * qB;
            grad[1][d] = c1A * qA + c1B * qB;
            grad[2][d] = c2A * qA + c2B * qB;
        }
    }
}

__global__ void k_mem_rest(ib_membrane m, const double* X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m.n && m.nbr_ptr) {
        double xi[3], xj[3], r[3];
        ld3(X, m.n, i, xi);
        for (int e = m.nbr_ptr[i]; e < m.nbr_ptr[i + 1]; ++e) {
            ld3(X, m.n, m.nbr_idx[e], xj);
            sub(xj, xi, r);
            m.rest_len[e] = sqrt(dt3(r, r));
        }
    }
    if (i < m.nh) {
        double x[4][3], gdummy[4][3], c, sn;
        for (int k = 0; k < 4; ++k) ld3(X, m.n, m.hinges[4 * i + k], x[k]);
        hinge(x, gdummy, false, c, sn);
        m.rest_cs[2 * i] = c;
        m.rest_cs[2 * i + 1] = sn;
    }
}

// Bending force of a hinge on one of its vertices (role 0..3): -k_b sin(theta - theta0) times
// that vertex's row of grad(theta) (the rows of `hinge`), computed for that row alone.
__device__ __forceinline__ void hinge_role_force(const double x[4][3], int role, double c0, double s0, double kb,
                                                 double out[3]) {
    double a[3], b[3], nA[3], nB[3], e[3], cr[3];
    sub(x[1], x[0], a); sub(x[2], x[0], b); crs(a, b, nA);
    sub(x[2], x[3], a); sub(x[1], x[3], b); crs(a, b, nB);
    sub(x[2], x[1], e);
    const double AA = dt3(nA, nA), BB = dt3(nB, nB), L = sqrt(dt3(e, e));
    const double iab = 1.0 / sqrt(AA * BB), iL = 1.0 / L;
    crs(nA, nB, cr);
    const double cth = dt3(nA, nB) * iab;
    const double sth = dt3(cr, e) * iab * iL;
    const double dE = kb * (sth * c0 - cth * s0);
    double cA, cB;
    if (role == 0) {
        cA = -L;
        cB = 0.0;
    } else if (role == 3) {
        cA = 0.0;
        cB = -L;
    } else {
        // role 1: -((x0 - x2).e, (x3 - x2).e)/|e|; role 2: ((x0 - x1).e, (x3 - x1).e)/|e|
        const int o = role == 1 ? 2 : 1;
        const double sg = role == 1 ? -iL : iL;
        double t0[3], t3[3];
        sub(x[0], x[o], t0);
        sub(x[3], x[o], t3);
        cA = sg * dt3(t0, e);
        cB = sg * dt3(t3, e);
    }
    const double qa = cA / AA, qb = cB / BB;
    for (int d = 0; d < 3; ++d) out[d] = -dE * (qa * nA[d] + qb * nB[d]);
}

// ---------------------------------------------------------------- area and volume (Eq. (4)-(5))
__host__ __device__ inline bool constraints_on(const ib_membrane& m) {
    return m.tri && m.nt > 0 && m.nb > 0 && (m.k_area_global != 0.0 || m.k_area_local != 0.0 || m.k_volume != 0.0);
}

// Per body (one workgroup of BODY_THREADS): S^total = sum of the triangle areas |n|/2 with
// n = (b - a) x (c - a), and V = sum of a.(b x c)/6 over its outward triangles (divergence
// theorem), as strided partial sums and a fixed tree, so they do not depend on scheduling.
// out[4b..4b+1] = S^total, V; with coef, also out[4b+2..4b+3] = the force coefficients
// k_s (S^total - S_0^total)/S_0^total and k_v (V - V_0)/V_0 (rest values in m.rest_body).
constexpr int BODY_THREADS = 256;
__device__ __forceinline__ void body_block(const ib_membrane& m, const double* X, double* out, int64_t b,
                                           bool coef) {
    __shared__ double sa[BODY_THREADS], sv[BODY_THREADS];
    double S = 0.0, V6 = 0.0;
#pragma unroll 4
    for (int64_t t = m.body_tri[b] + threadIdx.x; t < m.body_tri[b + 1]; t += BODY_THREADS) {
        double p[3][3], u[3], v[3], nn[3], bc[3];
        for (int k = 0; k < 3; ++k) ld3(X, m.n, m.tri[3 * t + k], p[k]);
        sub(p[1], p[0], u);
        sub(p[2], p[0], v);
        crs(u, v, nn);
        S += 0.5 * sqrt(dt3(nn, nn));
        crs(p[1], p[2], bc);
        V6 += dt3(p[0], bc);
    }
    sa[threadIdx.x] = S;
    sv[threadIdx.x] = V6;
    __syncthreads();
    for (int w = BODY_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sv[threadIdx.x] += sv[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double St = sa[0], V = sv[0] / 6.0;
        if (coef) {
            out[4 * b] = St;
            out[4 * b + 1] = V;
            out[4 * b + 2] = m.k_area_global * (St - m.rest_body[2 * b]) / m.rest_body[2 * b];
            out[4 * b + 3] = m.k_volume * (V - m.rest_body[2 * b + 1]) / m.rest_body[2 * b + 1];
        } else {
            out[2 * b] = St;
            out[2 * b + 1] = V;
        }
    }
}

__global__ void __launch_bounds__(BODY_THREADS) k_mem_bodies(ib_membrane m, const double* X, double* out, bool coef) {
    body_block(m, X, out, blockIdx.x, coef);
}

// Rest area S_0 of each triangle.
__global__ void k_tri_rest(ib_membrane m, const double* X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.nt) return;
    double p[3][3], u[3], v[3], nn[3];
    for (int k = 0; k < 3; ++k) ld3(X, m.n, m.tri[3 * t + k], p[k]);
    sub(p[1], p[0], u);
    sub(p[2], p[0], v);
    crs(u, v, nn);
    m.rest_area[t] = 0.5 * sqrt(dt3(nn, nn));
}

// ---------------------------------------------------------------- FE bending (Eq. (6)-(10))
__host__ __device__ inline bool fe_on(const ib_membrane& m) { return m.elem6 && m.ne > 0 && m.k_fe != 0.0; }

// Scratch layout (CSR order of the element-node incidences, nnz = 6 ne): per incidence the
// symmetric curvature tensor (xx, yy, zz, xy, xz, yz), the unit normal and the area share (10),
// then the surface gradient of K (3), then the surface divergence of grad K (1); per node K, G,
// the averaged unit normal and the area (6).
struct FeWork {
    double *kap, *grad, *div, *node;
};
__device__ __forceinline__ FeWork fe_work(const ib_membrane& m) {
    const int64_t nnz = 6 * m.ne;
    return {m.fe_work, m.fe_work + 10 * nnz, m.fe_work + 13 * nnz, m.fe_work + 14 * nnz};
}

// Parametric position (xi, eta) of local node k: corners (0,0), (1,0), (0,1), then the midpoints
// (1/2,0), (1/2,1/2), (0,1/2).
__device__ __forceinline__ void fe_node_xi(int k, double& xi, double& eta) {
    xi = (k == 1) ? 1.0 : ((k == 3 || k == 4) ? 0.5 : 0.0);
    eta = (k == 2) ? 1.0 : ((k == 4 || k == 5) ? 0.5 : 0.0);
}

// d N_j / d xi and d N_j / d eta of the quadratic six-node basis at (xi, eta); with z = 1 - xi - eta
// the basis is z(2z-1), xi(2xi-1), eta(2eta-1), 4 xi z, 4 xi eta, 4 eta z.
__device__ __forceinline__ void fe_dbasis(double xi, double eta, double dx[6], double de[6]) {
    const double z = 1.0 - xi - eta;
    dx[0] = 1.0 - 4.0 * z;  de[0] = 1.0 - 4.0 * z;
    dx[1] = 4.0 * xi - 1.0; de[1] = 0.0;
    dx[2] = 0.0;            de[2] = 4.0 * eta - 1.0;
    dx[3] = 4.0 * (z - xi); de[3] = -4.0 * xi;
    dx[4] = 4.0 * eta;      de[4] = 4.0 * xi;
    dx[5] = -4.0 * eta;     de[5] = 4.0 * (z - eta);
}

// Geometry of the interpolated surface of an element (node positions P) at its local node k:
// tangents a1 = dX/dxi, a2 = dX/deta, |a1 x a2|, unit normal n, dual tangents d1, d2
// (d_a . a_b = delta_ab, in the tangent plane) and with `curv` the normal's derivatives
// dn/dxi, dn/deta (from the constant second derivatives of the quadratic interpolation).
struct FeFrame {
    double a1[3], a2[3], n[3], d1[3], d2[3], dn1[3], dn2[3], mn;
};
__device__ void fe_frame(const double P[6][3], int k, bool curv, FeFrame& f) {
    double xi, eta, dx[6], de[6];
    fe_node_xi(k, xi, eta);
    fe_dbasis(xi, eta, dx, de);
    for (int c = 0; c < 3; ++c) {
        double s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < 6; ++j) {
            s1 += dx[j] * P[j][c];
            s2 += de[j] * P[j][c];
        }
        f.a1[c] = s1;
        f.a2[c] = s2;
    }
    double m[3];
    crs(f.a1, f.a2, m);
    f.mn = sqrt(dt3(m, m));
    const double im = 1.0 / f.mn;
    for (int c = 0; c < 3; ++c) f.n[c] = m[c] * im;
    const double g11 = dt3(f.a1, f.a1), g12 = dt3(f.a1, f.a2), g22 = dt3(f.a2, f.a2);
    const double idet = 1.0 / (g11 * g22 - g12 * g12);
    for (int c = 0; c < 3; ++c) {
        f.d1[c] = (g22 * f.a1[c] - g12 * f.a2[c]) * idet;
        f.d2[c] = (g11 * f.a2[c] - g12 * f.a1[c]) * idet;
    }
    if (!curv) return;
    // second derivatives: X_xixi = 4(a + b) - 8 m_ab, X_xieta = 4(a - m_ab + m_bc - m_ca),
    // X_etaeta = 4(a + c) - 8 m_ca
    double a11[3], a12[3], a22[3];
    for (int c = 0; c < 3; ++c) {
        a11[c] = 4.0 * (P[0][c] + P[1][c]) - 8.0 * P[3][c];
        a12[c] = 4.0 * (P[0][c] - P[3][c] + P[4][c] - P[5][c]);
        a22[c] = 4.0 * (P[0][c] + P[2][c]) - 8.0 * P[5][c];
    }
    // d(a1 x a2)/dxi = a11 x a2 + a1 x a12, d(a1 x a2)/deta = a12 x a2 + a1 x a22; the unit
    // normal's derivative is the tangential part over |a1 x a2|
    double u[3], v[3], dm1[3], dm2[3];
    crs(a11, f.a2, u); crs(f.a1, a12, v);
    for (int c = 0; c < 3; ++c) dm1[c] = u[c] + v[c];
    crs(a12, f.a2, u); crs(f.a1, a22, v);
    for (int c = 0; c < 3; ++c) dm2[c] = u[c] + v[c];
    const double p1 = dt3(f.n, dm1), p2 = dt3(f.n, dm2);
    for (int c = 0; c < 3; ++c) {
        f.dn1[c] = (dm1[c] - p1 * f.n[c]) * im;
        f.dn2[c] = (dm2[c] - p2 * f.n[c]) * im;
    }
}

__device__ __forceinline__ void fe_load(const ib_membrane& m, const double* X, int64_t e, double P[6][3]) {
    for (int j = 0; j < 6; ++j) ld3(X, m.n, m.elem6[6 * e + j], P[j]);
}

__device__ __forceinline__ double tri_area(const double a[3], const double b[3], const double c[3]) {
    double u[3], v[3], w[3];
    sub(b, a, u);
    sub(c, a, v);
    crs(u, v, w);
    return 0.5 * sqrt(dt3(w, w));
}

// First pass, one element node per lane (8 lanes per element, 6 in use): Eq. (9)'s curvature
// tensor kappa = d1 (x) dn/dxi + d2 (x) dn/deta (symmetric part), the normal, and the node's area
// share: a third of the flat sub-triangles (a, m_ab, m_ca), (m_ab, b, m_bc), (m_ca, m_bc, c),
// (m_ab, m_bc, m_ca) that contain it.
__device__ __forceinline__ void fe_kappa_one(const ib_membrane& m, const double* X, int64_t t) {
    const int64_t e = t >> 3;
    const int k = (int)(t & 7);
    if (e >= m.ne || k >= 6) return;
    double P[6][3];
    fe_load(m, X, e, P);
    FeFrame f;
    fe_frame(P, k, true, f);
    double* o = fe_work(m).kap + 10 * (int64_t)m.elem_slot[6 * e + k];
    o[0] = f.d1[0] * f.dn1[0] + f.d2[0] * f.dn2[0];
    o[1] = f.d1[1] * f.dn1[1] + f.d2[1] * f.dn2[1];
    o[2] = f.d1[2] * f.dn1[2] + f.d2[2] * f.dn2[2];
    o[3] = 0.5 * (f.d1[0] * f.dn1[1] + f.d2[0] * f.dn2[1] + f.d1[1] * f.dn1[0] + f.d2[1] * f.dn2[0]);
    o[4] = 0.5 * (f.d1[0] * f.dn1[2] + f.d2[0] * f.dn2[2] + f.d1[2] * f.dn1[0] + f.d2[2] * f.dn2[0]);
    o[5] = 0.5 * (f.d1[1] * f.dn1[2] + f.d2[1] * f.dn2[2] + f.d1[2] * f.dn1[1] + f.d2[2] * f.dn2[1]);
    o[6] = f.n[0];
    o[7] = f.n[1];
    o[8] = f.n[2];
    double A;
    if (k < 3) {  // corner: its one sub-triangle
        const int mprev = k == 0 ? 5 : k + 2, mnext = k + 3;
        A = tri_area(P[k], P[mnext], P[mprev]);
    } else {      // midpoint: the centre sub-triangle and the two corner ones beside it
        const int c0 = k - 3, c1 = (k - 2) % 3;
        A = tri_area(P[3], P[4], P[5]) + tri_area(P[c0], P[k], P[c0 == 0 ? 5 : c0 + 2]) +
            tri_area(P[c1], P[c1 + 3], P[k]);
    }
    o[9] = A * (1.0 / 3.0);
}

__global__ void __launch_bounds__(256) k_fe_kappa(ib_membrane m, const double* X) {
    fe_kappa_one(m, X, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Node averages of the first pass for node i: K = tr(kappa)/2, G = ((tr kappa)^2 - tr(kappa^2))/2,
// the unit normal, the area.
__device__ __forceinline__ void fe_node_avg(const ib_membrane& m, int64_t i, double out[6]) {
    const double* w = fe_work(m).kap;
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int p0 = m.elem_ptr[i], p1 = m.elem_ptr[i + 1];
    for (int p = p0; p < p1; ++p)
        for (int q = 0; q < 10; ++q) s[q] += w[10 * (int64_t)p + q];
    const double ic = 1.0 / (double)(p1 - p0);
    double kap[6];
    for (int q = 0; q < 6; ++q) kap[q] = s[q] * ic;
    const double tr = kap[0] + kap[1] + kap[2];
    const double sq = kap[0] * kap[0] + kap[1] * kap[1] + kap[2] * kap[2] +
                      2.0 * (kap[3] * kap[3] + kap[4] * kap[4] + kap[5] * kap[5]);
    const double nl = 1.0 / sqrt(s[6] * s[6] + s[7] * s[7] + s[8] * s[8]);
    out[0] = 0.5 * tr;
    out[1] = 0.5 * (tr * tr - sq);
    out[2] = s[6] * nl;
    out[3] = s[7] * nl;
    out[4] = s[8] * nl;
    out[5] = s[9];
}

// Second pass: node averages of the first (stored once per node, by the node's first incidence),
// then at every element node the surface gradient of the quadratically interpolated K:
// d1 dK/dxi + d2 dK/deta.  The element's six lanes exchange their nodes' K by lane shuffles.
__global__ void __launch_bounds__(256) k_fe_grad(ib_membrane m, const double* X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t >> 3;
    const int k = (int)(t & 7);
    const bool on = e < m.ne && k < 6;
    const FeWork W = fe_work(m);
    double K = 0.0;
    if (on) {
        const int64_t i = m.elem6[6 * e + k];
        double nd[6];
        fe_node_avg(m, i, nd);
        K = nd[0];
        if (m.elem_slot[6 * e + k] == m.elem_ptr[i])
            for (int q = 0; q < 6; ++q) W.node[6 * i + q] = nd[q];
    }
    const int base = threadIdx.x & ~7;  // first lane of this element's group
    double Kj[6];
    for (int j = 0; j < 6; ++j) Kj[j] = __shfl(K, base + j, 64);
    if (!on) return;
    double P[6][3];
    fe_load(m, X, e, P);
    FeFrame f;
    fe_frame(P, k, false, f);
    double xi, eta, dx[6], de[6];
    fe_node_xi(k, xi, eta);
    fe_dbasis(xi, eta, dx, de);
    double k1 = 0.0, k2 = 0.0;
    for (int j = 0; j < 6; ++j) {
        k1 += dx[j] * Kj[j];
        k2 += de[j] * Kj[j];
    }
    double* o = W.grad + 3 * (int64_t)m.elem_slot[6 * e + k];
    for (int c = 0; c < 3; ++c) o[c] = f.d1[c] * k1 + f.d2[c] * k2;
}

// Third pass: node averages of the gradient, then at every element node the surface divergence
// d1 . d(grad K)/dxi + d2 . d(grad K)/deta of the interpolated gradient field.
__global__ void __launch_bounds__(256) k_fe_div(ib_membrane m, const double* X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t >> 3;
    const int k = (int)(t & 7);
    const bool on = e < m.ne && k < 6;
    const FeWork W = fe_work(m);
    double g[3] = {0.0, 0.0, 0.0};
    if (on) {
        const int64_t i = m.elem6[6 * e + k];
        const int p0 = m.elem_ptr[i], p1 = m.elem_ptr[i + 1];
        for (int p = p0; p < p1; ++p)
            for (int c = 0; c < 3; ++c) g[c] += W.grad[3 * (int64_t)p + c];
        const double ic = 1.0 / (double)(p1 - p0);
        for (int c = 0; c < 3; ++c) g[c] *= ic;
    }
    const int base = threadIdx.x & ~7;
    double G[6][3];
    for (int j = 0; j < 6; ++j)
        for (int c = 0; c < 3; ++c) G[j][c] = __shfl(g[c], base + j, 64);
    if (!on) return;
    double P[6][3];
    fe_load(m, X, e, P);
    FeFrame f;
    fe_frame(P, k, false, f);
    double xi, eta, dx[6], de[6];
    fe_node_xi(k, xi, eta);
    fe_dbasis(xi, eta, dx, de);
    double g1[3] = {0.0, 0.0, 0.0}, g2[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 6; ++j)
        for (int c = 0; c < 3; ++c) {
            g1[c] += dx[j] * G[j][c];
            g2[c] += de[j] * G[j][c];
        }
    W.div[m.elem_slot[6 * e + k]] = dt3(f.d1, g1) + dt3(f.d2, g2);
}

// Inverse of the node -> element-node incidence CSR: position of (element, local node).
__global__ void k_fe_slots(ib_membrane m, int64_t nnz) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) {
        const int32_t code = m.elem_inc[p];
        m.elem_slot[6 * (int64_t)(code >> 3) + (code & 7)] = (int32_t)p;
    }
}

// Per node (NODE_LANES lanes each, partial sums combined by a fixed butterfly): springs (CSR), the
// bending forces of the hinges it belongs to, the area and volume constraints of its
// triangles, tether.
// For the corner a of triangle (a, b, c) (any cyclic order), with n = (b - a) x (c - a):
//   dS/da = n_hat x (c - b) / 2,  dV/da = (b x c) / 6,
//   F_a -= [k_s (S^total - S_0^total)/S_0^total + k_t (S - S_0)/S_0] dS/da + k_v (V - V_0)/V_0 dV/da.  In the coupled step (rec != NULL) it also puts F
// into the node records and the workgroup's max |F| into bmax[workgroup], the two parts of
// the binning that need F.
// CONS: the constraint loop is compiled in (only launched when constraints_on(m)), so the
// plain membrane keeps the smaller register footprint.
template <bool CONS>
__device__ __forceinline__ void forces_block(const ib_membrane& m, const double* X, float* Fout, float* rec,
                                             uint32_t* bmax, int64_t blk, const IbArgs* ia = nullptr) {
    const int64_t i = (blk * blockDim.x + threadIdx.x) / NODE_LANES;
    const int sl = threadIdx.x & (NODE_LANES - 1);
    const bool valid = i < m.n;
    double xi[3] = {0.0, 0.0, 0.0}, xj[3], r[3], F[3] = {0.0, 0.0, 0.0};
    if (valid) ld3(X, m.n, i, xi);
    if (valid && m.nbr_ptr) {
        for (int e = m.nbr_ptr[i] + sl; e < m.nbr_ptr[i + 1]; e += NODE_LANES) {
            ld3(X, m.n, m.nbr_idx[e], xj);
            sub(xj, xi, r);
            const double len = sqrt(dt3(r, r));
            const double s = m.k_spring * (len - m.rest_len[e]) / len;
            F[0] += s * r[0]; F[1] += s * r[1]; F[2] += s * r[2];
        }
    }
    if (valid && m.hinge_ptr && m.k_bend != 0.0) {
        // the node evaluates each hinge it belongs to for its own role
        for (int e = m.hinge_ptr[i] + sl; e < m.hinge_ptr[i + 1]; e += NODE_LANES) {
            const int32_t code = m.hinge_inc[e];
            const int64_t h = code >> 2;
            double x[4][3], g[3];
            for (int k = 0; k < 4; ++k) ld3(X, m.n, m.hinges[4 * h + k], x[k]);
            hinge_role_force(x, code & 3, m.rest_cs[2 * h], m.rest_cs[2 * h + 1], m.k_bend, g);
            F[0] += g[0]; F[1] += g[1]; F[2] += g[2];
        }
    }
    if (CONS && valid) {
        for (int e = m.tri_ptr[i] + sl; e < m.tri_ptr[i + 1]; e += NODE_LANES) {
            const int32_t code = m.tri_inc[e];
            const int64_t t = code >> 2;
            const int k = code & 3;
            double pa[3], pb[3], pc[3], u[3], v[3], nn[3], ed[3], dS[3], dV[3];
            ld3(X, m.n, m.tri[3 * t + k], pa);
            ld3(X, m.n, m.tri[3 * t + (k + 1) % 3], pb);
            ld3(X, m.n, m.tri[3 * t + (k + 2) % 3], pc);
            sub(pb, pa, u);
            sub(pc, pa, v);
            crs(u, v, nn);
            const double nl = sqrt(dt3(nn, nn));  // |n| = 2 S
            const int bd = m.tri_body[t];
            const double ct = m.k_area_local * (0.5 * nl - m.rest_area[t]) / m.rest_area[t];
            // (cs + ct) dS/da with dS/da = n x (c - b) / (2 |n|); cv dV/da with dV/da = (b x c)/6
            const double al = (m.body_now[4 * bd + 2] + ct) * 0.5 / nl;
            const double be = m.body_now[4 * bd + 3] * (1.0 / 6.0);
            sub(pc, pb, ed);
            crs(nn, ed, dS);
            crs(pb, pc, dV);
            for (int d = 0; d < 3; ++d) F[d] -= al * dS[d] + be * dV[d];
        }
    }
    // adhesion bonds (Eq. (14)): each bonded receptor of the node's incidences pulls with the
    // spring force times the node's barycentric weight
    if (m.adh_nr > 0 && valid) {
        for (int e = m.rec_ptr[i] + sl; e < m.rec_ptr[i + 1]; e += NODE_LANES) {
            const int32_t code = m.rec_inc[e];
            const int64_t rr = code >> 2;
            const int32_t l = m.bond[rr];
            if (l < 0) continue;
            double xr[3];
            for (int c = 0; c < 3; ++c) {
                double sacc = 0.0;
                for (int k = 0; k < 3; ++k) sacc += m.rec_bary[3 * rr + k] * X[c * m.n + m.rec_tri[3 * rr + k]];
                xr[c] = sacc;
            }
            double dx = xr[0] - m.lig_xz[2 * l], dz = xr[2] - m.lig_xz[2 * l + 1];
            dx -= m.adh_nx * rint(dx / m.adh_nx);
            dz -= m.adh_nz * rint(dz / m.adh_nz);
            const double dy = xr[1] - m.adh_wall_y;
            const double L = sqrt(dx * dx + dy * dy + dz * dz);
            const double f = -m.adh_sigma * (L - m.adh_lb) / L * m.rec_bary[3 * rr + (code & 3)];
            F[0] += f * dx;
            F[1] += f * dy;
            F[2] += f * dz;
        }
    }
    // FE bending: the node average of the third pass's divergence is Lap K
    double lap = 0.0;
    const bool fe = fe_on(m);
    if (fe && valid)
        for (int e = m.elem_ptr[i] + sl; e < m.elem_ptr[i + 1]; e += NODE_LANES) lap += fe_work(m).div[e];
#pragma unroll
    for (int d = 1; d < NODE_LANES; d <<= 1) {
        F[0] += __shfl_xor(F[0], d, 64);
        F[1] += __shfl_xor(F[1], d, 64);
        F[2] += __shfl_xor(F[2], d, 64);
        if (fe) lap += __shfl_xor(lap, d, 64);
    }
    if (fe && valid) {
        const double* nd = fe_work(m).node + 6 * i;
        const double K = nd[0];
        lap /= (double)(m.elem_ptr[i + 1] - m.elem_ptr[i]);
        const double f = 0.5 * m.k_fe * (lap + 2.0 * K * (K * K - nd[1])) * nd[5];
        for (int d = 0; d < 3; ++d) F[d] += f * nd[2 + d];
    }
    if (valid && m.anchors)
        for (int d = 0; d < 3; ++d) F[d] -= m.k_tether * (xi[d] - m.anchors[d * m.n + i]);
    float Ff[3] = {(float)F[0], (float)F[1], (float)F[2]};
    if (valid && sl == 0) {
        for (int d = 0; d < 3; ++d) Fout[d * m.n + i] = Ff[d];
        if (rec)
            for (int d = 0; d < 3; ++d) rec[i * REC + 16 + d] = Ff[d];
    }
    if (ia && ia->rec_in_forces && valid && sl < 3) {
        // a step between binnings: lane d writes axis d of the node's stencil base and weights
        // at X, and checks that the stencil is still inside the tiles the node was listed in
        const Chan& ch = ia->chan[ia->node_ch[i]];
        bool bad;
        record_axis(*ia, i, ch, sl, bad);
        const int4 lo = ia->nbin[2 * i], hi = ia->nbin[2 * i + 1];
        const int f = (int)floor(xi[sl]);
        const int l = sl == 0 ? lo.x : (sl == 1 ? lo.y : lo.z), h = sl == 0 ? hi.x : (sl == 1 ? hi.y : hi.z);
        if (bad) atomicOr(ia->flags, LBM_FLAG_NODE_OUTSIDE);
        if (f < l || f > h) atomicOr(ia->flags, LBM_FLAG_REBIN_MARGIN);
    }
    if (bmax) {
        // workgroup max |F| as float bits (NaN/Inf above every finite value), as the binning does
        float fm = 0.0f;
        if (valid)
            for (int d = 0; d < 3; ++d) {
                fm = fmaxf(fm, fabsf(Ff[d]));
                if (!isfinite(Ff[d])) fm = __uint_as_float(0x7f800000u);
            }
        uint32_t ub = __float_as_uint(fm);
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t o = __shfl_xor(ub, d, 64);
            ub = o > ub ? o : ub;
        }
        __shared__ uint32_t wm[16];
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = ub;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t mx = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) mx = wm[k] > mx ? wm[k] : mx;
            bmax[blk] = mx;
        }
    }
}

template <bool CONS>
__global__ void __launch_bounds__(256) k_mem_forces(ib_membrane m, const double* X, float* Fout) {
    forces_block<CONS>(m, X, Fout, nullptr, nullptr, blockIdx.x);
}

// The coupled step's second launch: the scan of the tile lists (workgroup 0, on binning steps;
// it needs only the binning) and the membrane forces (the rest, FS_THREADS / NODE_LANES nodes each),
// which also fill in the records' F and max |F| per workgroup, and between binnings the records'
// stencil bases and weights.
// 512 threads: node-force workgroups of 32 nodes spread over more CUs, while the scan
// workgroup still covers a few hundred flagged tiles per pass (on the 3,600-tile batch 1024 is
// 0.4% faster per step)
constexpr int FS_THREADS = 512;
template <bool CONS>
__global__ void __launch_bounds__(FS_THREADS) k_forces_scan(ib_membrane m, const double* X, float* F, IbArgs a) {
    if (blockIdx.x == 0) {
        if (a.do_scan) scan_block(a, false);
    } else {
        forces_block<CONS>(m, X, F, a.rec, a.blkmax, (int64_t)blockIdx.x - 1, &a);
    }
}

// The coupled step's first launch: the binning of the nodes by position (workgroups
// [0, nbb), dispatched first: theirs is the longer dependent chain), the bodies' areas and
// volumes for the constraints (the next nbd, one per body) and the first pass of the FE bending
// (the rest); the binning depends on neither.
template <bool CONS>
__global__ void __launch_bounds__(256) k_bin_first(ib_membrane m, const double* X, IbArgs a, int64_t nbb,
                                                   int64_t nbd) {
    const int64_t blk = blockIdx.x;
    if (blk < nbb) {
        bin_block(a, blk, false);
    } else if (CONS && blk < nbb + nbd) {
        body_block(m, X, m.body_now, blk - nbb, true);
    } else {
        fe_kappa_one(m, X, (blk - nbb - nbd) * blockDim.x + threadIdx.x);
    }
}

hipError_t launch_membrane_rest(const ib_membrane* m, const double* X_rest, hipStream_t s) {
    const int64_t n = m->n > m->nh ? m->n : m->nh;
    if (n <= 0) return hipSuccess;
    k_mem_rest<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(*m, X_rest);
    if (m->tri && m->nt > 0 && m->nb > 0) {
        k_tri_rest<<<dim3((unsigned)((m->nt + 255) / 256)), dim3(256), 0, s>>>(*m, X_rest);
        k_mem_bodies<<<dim3((unsigned)m->nb), dim3(BODY_THREADS), 0, s>>>(*m, X_rest, m->rest_body, false);
    }
    if (fe_on(*m)) {
        const int64_t nnz = 6 * m->ne;
        k_fe_slots<<<dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s>>>(*m, nnz);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_adhesion_setup(m, s);
    return e;
}

// The second and third FE bending passes (the first shares a launch or runs before them).
static void launch_fe_passes(const ib_membrane* m, const double* X, hipStream_t s) {
    const dim3 g((unsigned)((8 * m->ne + 255) / 256)), b(256);
    k_fe_grad<<<g, b, 0, s>>>(*m, X);
    k_fe_div<<<g, b, 0, s>>>(*m, X);
}

hipError_t launch_membrane_forces(const ib_membrane* m, const double* X, float* F, hipStream_t s) {
    if (m->n <= 0) return hipSuccess;
    if (fe_on(*m)) {
        k_fe_kappa<<<dim3((unsigned)((8 * m->ne + 255) / 256)), dim3(256), 0, s>>>(*m, X);
        launch_fe_passes(m, X, s);
    }
    const dim3 gf((unsigned)((NODE_LANES * m->n + 255) / 256)), bf(256);
    if (constraints_on(*m)) {
        k_mem_bodies<<<dim3((unsigned)m->nb), dim3(BODY_THREADS), 0, s>>>(*m, X, m->body_now, true);
        k_mem_forces<true><<<gf, bf, 0, s>>>(*m, X, F);
    } else {
        k_mem_forces<false><<<gf, bf, 0, s>>>(*m, X, F);
    }
    return hipGetLastError();
}

// Coupled step, forces to node lists: [binning | body sums | FE first pass] -> [scan | membrane forces] ->
// scatter (whose first workgroup sets the spread's scale from the forces).
hipError_t launch_forces_scatter(lbm_ctx* c, const ib_membrane* m, const double* X, float* F, IbArgs& a, bool bin) {
    const int64_t nbb = bin ? (a.n + 255) / 256 : 0;
    const int64_t nbd = constraints_on(*m) ? m->nb : 0;
    const int64_t nbe = fe_on(*m) ? (8 * m->ne + 255) / 256 : 0;
    const dim3 g1((unsigned)(nbb + nbd + nbe));
    if (nbd > 0)
        k_bin_first<true><<<g1, dim3(256), 0, c->stream>>>(*m, X, a, nbb, nbd);
    else if (nbb + nbe > 0)
        k_bin_first<false><<<g1, dim3(256), 0, c->stream>>>(*m, X, a, nbb, 0);
    if (nbe > 0) launch_fe_passes(m, X, c->stream);
    const int64_t nbf = (NODE_LANES * m->n + FS_THREADS - 1) / FS_THREADS;
    a.blkmax_n = nbf;
    a.scale_in_scatter = a.scale_local ? 0 : 1;
    a.do_scan = bin ? 1 : 0;
    a.rec_in_forces = bin ? 0 : 1;
    if (nbd > 0)
        k_forces_scan<true><<<dim3((unsigned)(1 + nbf)), dim3(FS_THREADS), 0, c->stream>>>(*m, X, F, a);
    else
        k_forces_scan<false><<<dim3((unsigned)(1 + nbf)), dim3(FS_THREADS), 0, c->stream>>>(*m, X, F, a);
    if (bin) {
        const int64_t nbs = nbb > 0 ? nbb : 1;  // the first workgroup sets the scale, also with no nodes
        k_ib_scatter<<<dim3((unsigned)nbs), dim3(256), 0, c->stream>>>(a);
    }
    return hipGetLastError();
}


}  // namespace lbmib
