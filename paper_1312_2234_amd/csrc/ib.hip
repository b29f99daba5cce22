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
constexpr int HS = 2048;   // hash entries per block
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

__global__ void __launch_bounds__(256) k_ib_bin(IbArgs a) {
    __shared__ int hkey[HS];
    __shared__ int hcnt[HS];
    __shared__ float wmax[4];
    for (int e = threadIdx.x; e < HS; e += blockDim.x) {
        hkey[e] = -1;
        hcnt[e] = 0;
    }
    __syncthreads();
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float fm = 0.0f;
    if (m < a.n) {
        const int c = a.node_ch[m];
        const Chan& ch = a.chan[c];
        float* r = a.rec + m * REC;
        float w[3][4];
        int b[3];
        bool bad = false;
        for (int d = 0; d < 3; ++d) {
            const double X = a.X[d * a.n + m];
            const int dim = d == 0 ? ch.nx : (d == 1 ? ch.ny : ch.nz);
            const bool finite = isfinite(X) && fabs(X) < 1e9;
            int64_t base = finite ? ib_weights(a.kernel, X, w[d]) : 0;
            if (!finite) {
                bad = true;
                w[d][0] = w[d][1] = w[d][2] = w[d][3] = 0.0f;
            }
            if (d == 1 && ch.walls) {
                if (base < -2 || base > ch.ny - 2) bad = true;  // node outside y in [-1, ny)
                if (base < -4) base = -4;
                if (base > ch.ny) base = ch.ny;
                b[d] = (int)base;
            } else {
                b[d] = wrapi(base, dim);
            }
        }
        if (bad) atomicOr(a.flags, LBM_FLAG_NODE_OUTSIDE);
        r[0] = __int_as_float(b[0]);
        r[1] = __int_as_float(b[1]);
        r[2] = __int_as_float(b[2]);
        r[3] = __int_as_float(c);
        for (int k = 0; k < 4; ++k) {
            r[4 + k] = w[0][k];
            r[8 + k] = w[1][k];
            r[12 + k] = w[2][k];
        }
        for (int d = 0; d < 3; ++d) {
            const float F = a.F[d * a.n + m];
            r[16 + d] = F;
            fm = fmaxf(fm, fabsf(F));
            if (!isfinite(F)) fm = __uint_as_float(0x7f800000u);
        }
        int32_t* rk = a.rank + m * MAXT;
        for_tiles(ch, b[0], b[1], b[2], [&](int q, int64_t T) {
            int h = (int)(((uint32_t)T * 2654435761u) >> 21) & (HS - 1);
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
        });
    }
    // block maximum of |F| (NaN/Inf bits compare above all finite values)
    uint32_t ub = __float_as_uint(fm);
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(ub, d, 64);
        ub = o > ub ? o : ub;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = __uint_as_float(ub);
    __syncthreads();
    int32_t* bb = a.blkbase + (int64_t)blockIdx.x * HS;
    for (int e = threadIdx.x; e < HS; e += blockDim.x) {
        const int T = hkey[e];
        int base = 0;
        if (T >= 0) {
            base = atomicAdd(&a.set.cnt[T], hcnt[e]);
            if (base == 0) append_flagged(a, T);
        }
        bb[e] = base;
    }
    if (threadIdx.x == 0) {
        uint32_t mx = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            const uint32_t v = __float_as_uint(wmax[k]);
            mx = v > mx ? v : mx;
        }
        atomicMax(&a.set.hdr->fmax_bits, mx);
    }
}

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

__global__ void __launch_bounds__(1024) k_ib_scan(IbArgs a) {
    __shared__ int wsum[16];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // clear the tile set used by the spread before last
    const int nfo = a.other.hdr->nflag;
    for (int k = tid; k < nfo; k += blockDim.x) {
        const int T = a.other.flag_list[k];
        a.other.cnt[T] = 0;
        a.other.tile_slot[T] = -1;
    }
    const int nf = a.set.hdr->nflag;
    if (tid == 0) carry = 0;
    __syncthreads();  // every thread has read the other set's count before it is reset below
    for (int base = 0; base < nf; base += blockDim.x) {
        const int k = base + tid;
        const int v = k < nf ? a.set.cnt[a.set.flag_list[k]] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            const int nw = blockDim.x >> 6;
            int x = lane < nw ? wsum[lane] : 0;
            x = wave_incl_scan(x);
            if (lane < nw) wsum[lane] = x;
        }
        __syncthreads();
        const int excl = carry + (wave ? wsum[wave - 1] : 0) + incl - v;
        if (k < nf) {
            a.set.slot_off[k] = excl;
            a.set.tile_slot[a.set.flag_list[k]] = k;
        }
        __syncthreads();
        if (tid == blockDim.x - 1) carry = excl + v;
        __syncthreads();
    }
    if (tid == 0) {
        a.set.slot_off[nf] = carry;
        a.other.hdr->nflag = 0;
        a.other.hdr->fmax_bits = 0;
        a.other.hdr->nonfinite = 0;
        a.other.hdr->scale_exp = 0;
        // fixed-point scale: |contribution| <= max|F|/8 and at most n contributions per
        // cell, so |sum| < n * 2^e / 8 with max|F| < 2^e; keep sums below 2^62.
        const float fm = __uint_as_float(a.set.hdr->fmax_bits);
        int s = 0;
        if (!isfinite(fm)) {
            a.set.hdr->nonfinite = 1;
            atomicOr(a.flags, LBM_FLAG_FORCE_NONFINITE);
        } else if (fm > 0.0f) {
            int e;
            frexpf(fm, &e);  // fm < 2^e
            int L = 1;
            while ((1ll << L) < a.n) ++L;
            s = 62 - e - L;
        }
        a.set.hdr->scale_exp = s;
        if (carry > a.list_cap) atomicOr(a.flags, LBM_FLAG_LIST_OVERFLOW);
    }
}

// ---------------------------------------------------------------- scatter (no atomics)
__global__ void __launch_bounds__(256) k_ib_scatter(IbArgs a) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n) return;
    const float* r = a.rec + m * REC;
    const Chan& ch = a.chan[__float_as_int(r[3])];
    const int32_t* rk = a.rank + m * MAXT;
    const int32_t* bb = a.blkbase + (m >> 8) * HS;
    for_tiles(ch, __float_as_int(r[0]), __float_as_int(r[1]), __float_as_int(r[2]), [&](int q, int64_t T) {
        const int packed = rk[q];
        const int rr = packed >= 0 ? bb[packed >> 16] + (packed & 0xffff) : -packed - 1;
        const int slot = a.set.tile_slot[T];
        const int64_t pos = (int64_t)a.set.slot_off[slot] + rr;
        if (pos < a.list_cap) a.list[pos] = (int32_t)m;
    });
}

// ---------------------------------------------------------------- spread (LDS, fixed point)
// Work item = (flagged tile, one of its eight 4x4x4 sub-tiles): the tile's node list is
// scanned by all threads, each node adding its stencil points that fall in the sub-tile.
__global__ void __launch_bounds__(256) k_ib_spread(IbArgs a) {
    __shared__ unsigned long long acc[3 * 64];
    const int nf = a.set.hdr->nflag;
    const int sexp = a.set.hdr->scale_exp;
    const bool nonfinite = a.set.hdr->nonfinite != 0;
    const double scale = ldexp(1.0, sexp), inv = ldexp(1.0, -sexp);
    // the eight sub-tiles of a tile go to workgroups dealt to the same XCD (the dispatcher
    // deals workgroups round-robin over 8 XCDs), so the tile's node records stay in one L2
    const int b = blockIdx.x;
    const int first = (b & ~63) | ((b & 7) << 3) | ((b >> 3) & 7);
    for (int wi = first; wi < nf * 8; wi += gridDim.x) {
        const int slot = wi >> 3, sub = wi & 7;
        for (int k = threadIdx.x; k < 3 * 64; k += blockDim.x) acc[k] = 0ull;
        __syncthreads();
        const int T = a.set.flag_list[slot];
        const Chan& ch = a.chan[a.set.flag_ch[slot]];
        const int t = (int)(T - ch.tile_off);
        const int sx = (t % ch.tnx) * TILE + 4 * (sub & 1);
        const int sy = ((t / ch.tnx) % ch.tny) * TILE + 4 * ((sub >> 1) & 1);
        const int sz = (t / (ch.tnx * ch.tny)) * TILE + 4 * (sub >> 2);
        int64_t beg = a.set.slot_off[slot], end = a.set.slot_off[slot + 1];
        if (end > a.list_cap) end = a.list_cap;
        for (int64_t k = beg + threadIdx.x; k < end; k += blockDim.x) {
            const int64_t m = a.list[k];
            const float* r = a.rec + m * REC;
            Stencil s;
            stencil_cells(ch, __float_as_int(r[0]), __float_as_int(r[1]), __float_as_int(r[2]), s);
            uint32_t mx = 0, my = 0, mz = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                mx |= ((unsigned)(s.x[q] - sx) < 4u) << q;
                my |= (s.yok[q] && (unsigned)(s.y[q] - sy) < 4u) << q;
                mz |= ((unsigned)(s.z[q] - sz) < 4u) << q;
            }
            if (!mx || !my || !mz) continue;
            const float F0 = r[16], F1 = r[17], F2 = r[18];
            for (int cz4 = 0; cz4 < 4; ++cz4) {
                if (!((mz >> cz4) & 1)) continue;
                for (int cy4 = 0; cy4 < 4; ++cy4) {
                    if (!((my >> cy4) & 1)) continue;
                    const float wyz = r[8 + cy4] * r[12 + cz4];
                    for (int cx4 = 0; cx4 < 4; ++cx4) {
                        if (!((mx >> cx4) & 1)) continue;
                        const float ww = r[4 + cx4] * wyz;
                        const int loc = ((s.z[cz4] - sz) << 4) | ((s.y[cy4] - sy) << 2) | (s.x[cx4] - sx);
                        atomicAdd(&acc[loc], (unsigned long long)(long long)rint((double)(ww * F0) * scale));
                        atomicAdd(&acc[64 + loc], (unsigned long long)(long long)rint((double)(ww * F1) * scale));
                        atomicAdd(&acc[128 + loc], (unsigned long long)(long long)rint((double)(ww * F2) * scale));
                    }
                }
            }
        }
        __syncthreads();
        float* out = a.force + (int64_t)slot * (3 * TILE_CELLS);
        for (int k = threadIdx.x; k < 3 * 64; k += blockDim.x) {
            const int d = k >> 6, l = k & 63;
            const int lx = (sx & 7) + (l & 3), ly = (sy & 7) + ((l >> 2) & 3), lz = (sz & 7) + (l >> 4);
            out[d * TILE_CELLS + ((lz << 6) | (ly << 3) | lx)] =
                nonfinite ? __builtin_nanf("") : (float)((double)(long long)acc[k] * inv);
        }
        __syncthreads();
    }
}

hipError_t launch_ib_spread(lbm_ctx* c, const IbArgs& a) {
    const unsigned nb = (unsigned)((a.n + 255) / 256);
    if (a.n > 0) k_ib_bin<<<dim3(nb), dim3(256), 0, c->stream>>>(a);
    k_ib_scan<<<dim3(1), dim3(1024), 0, c->stream>>>(a);
    if (a.n > 0) k_ib_scatter<<<dim3(nb), dim3(256), 0, c->stream>>>(a);
    int64_t g = 8 * c->max_slots < 8192 ? 8 * c->max_slots : 8192;
    g = (g + 63) & ~int64_t(63);  // whole groups of 64 for the XCD-aware mapping
    k_ib_spread<<<dim3((unsigned)g), dim3(256), 0, c->stream>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- interpolation
// Fluid velocity of the current state, v = (j + (F_body + g)/2)/rho (Eq. (18) and the
// shift under Eq. (19)), on every cell of every flagged tile.
template <class St>
__global__ void __launch_bounds__(512) k_ib_vel(IbArgs a) {
    using T = typename St::T;
    const int nf = a.set.hdr->nflag;
    for (int slot = blockIdx.x; slot < nf; slot += gridDim.x) {
        const int T_ = a.set.flag_list[slot];
        const Chan& ch = a.chan[a.set.flag_ch[slot]];
        const int t = (int)(T_ - ch.tile_off);
        const int ox = (t % ch.tnx) * TILE, oy = ((t / ch.tnx) % ch.tny) * TILE, oz = (t / (ch.tnx * ch.tny)) * TILE;
        const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS);
        float* vb = a.vel + (int64_t)slot * (3 * TILE_CELLS);
        for (int l = threadIdx.x; l < TILE_CELLS; l += blockDim.x) {
            const int x = ox + (l & 7), y = oy + ((l >> 3) & 7), z = oz + (l >> 6);
            if (x >= ch.nx || y >= ch.ny || z >= ch.nz) continue;
            const int32_t n = x + ch.nx * (y + ch.ny * z);
            float g[Q];
            pull<St>((const T*)a.pop + ch.pop_off, ch, ch.ncell, n, x, y, z, g);
            float drho, jx, jy, jz;
            moments(g, drho, jx, jy, jz);
            const float ir = 1.0f / (1.0f + drho);
            vb[l] = (jx + 0.5f * (ch.body[0] + fb[l])) * ir;
            vb[TILE_CELLS + l] = (jy + 0.5f * (ch.body[1] + fb[TILE_CELLS + l])) * ir;
            vb[2 * TILE_CELLS + l] = (jz + 0.5f * (ch.body[2] + fb[2 * TILE_CELLS + l])) * ir;
        }
    }
}

// U_m = sum over the stencil of v(x) phi phi phi, rows inside a wall taking the wall
// velocity; optionally X_out = X + U.  Sixteen lanes per node: lane (b, c) takes stencil
// row y = base_y + b, z = base_z + c and its four x cells; the 16 partial sums are
// combined by a fixed butterfly, so the result does not depend on scheduling.
template <class St>
__global__ void __launch_bounds__(256) k_ib_gather(IbArgs a) {
    using T = typename St::T;
    // consecutive node blocks on the same XCD: neighbouring nodes share tiles in one L2
    const int64_t G = gridDim.x, bx = blockIdx.x, per = G >> 3, rem = G & 7, xcd = bx & 7;
    const int64_t L = xcd * per + (xcd < rem ? xcd : rem) + (bx >> 3);
    const int64_t m = (L * blockDim.x + threadIdx.x) >> 4;
    const int sl = threadIdx.x & 15, bq = sl & 3, cq = sl >> 2;
    float U[3] = {0.f, 0.f, 0.f};
    double X[3] = {0.0, 0.0, 0.0};
    const bool valid = m < a.n;
    if (valid) {
        const int c = a.node_ch[m];
        const Chan& ch = a.chan[c];
        float w[3][4];
        int b[3];
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
        Stencil s;
        stencil_cells(ch, b[0], b[1], b[2], s);
        const float wyz = w[1][bq] * w[2][cq];
        const int y = s.y[bq], z = s.z[cq];
#pragma unroll
        for (int ax = 0; ax < 4; ++ax) {
            const float ww = w[0][ax] * wyz;
            float v0, v1, v2;
            if (!s.yok[bq]) {
                const float* uw = y < 0 ? ch.uw_lo : ch.uw_hi;
                v0 = uw[0]; v1 = uw[1]; v2 = uw[2];
            } else {
                const int x = s.x[ax];
                const int slot = a.set.tile_slot[tile_of(ch, x, y, z)];
                if (slot >= 0) {
                    const float* vb = a.vel + (int64_t)slot * (3 * TILE_CELLS) + tile_local(x, y, z);
                    v0 = vb[0]; v1 = vb[TILE_CELLS]; v2 = vb[2 * TILE_CELLS];
                } else {  // not under any spread stencil: no IB force here
                    const int32_t n = x + ch.nx * (y + ch.ny * z);
                    float g[Q];
                    pull<St>((const T*)a.pop + ch.pop_off, ch, ch.ncell, n, x, y, z, g);
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
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
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
    int64_t g = c->max_slots < 4096 ? c->max_slots : 4096;
    if (g < 1) g = 1;
    k_ib_vel<St><<<dim3((unsigned)g), dim3(512), 0, c->stream>>>(a);
    if (a.n > 0) k_ib_gather<St><<<dim3((unsigned)((16 * a.n + 255) / 256)), dim3(256), 0, c->stream>>>(a);
}

hipError_t launch_ib_interp(lbm_ctx* c, const IbArgs& a) {
    switch (c->storage) {
        case LBM_STORE_F32: launch_interp_typed<StF32>(c, a); break;
        case LBM_STORE_F16: launch_interp_typed<StF16>(c, a); break;
        case LBM_STORE_BF16: launch_interp_typed<StBF16>(c, a); break;
    }
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
__device__ double hinge(const double x[4][3], double grad[4][3], bool want_grad) {
    double a[3], b[3], nA[3], nB[3], e[3], cr[3];
    sub(x[1], x[0], a); sub(x[2], x[0], b); crs(a, b, nA);
    sub(x[2], x[3], a); sub(x[1], x[3], b); crs(a, b, nB);
    sub(x[2], x[1], e);
    const double AA = dt3(nA, nA), BB = dt3(nB, nB), L = sqrt(dt3(e, e));
    const double la = sqrt(AA), lb = sqrt(BB);
    crs(nA, nB, cr);
    const double theta = atan2(dt3(cr, e) / (la * lb * L), dt3(nA, nB) / (la * lb));
    if (want_grad) {
        double t0[3], t3[3];
        sub(x[0], x[2], t0); sub(x[3], x[2], t3);
        const double c1A = -dt3(t0, e) / L, c1B = -dt3(t3, e) / L;
        sub(x[0], x[1], t0); sub(x[3], x[1], t3);
        const double c2A = dt3(t0, e) / L, c2B = dt3(t3, e) / L;
        for (int d = 0; d < 3; ++d) {
            const double qA = nA[d] / AA, qB = nB[d] / BB;
            grad[0][d] = -L * qA;
            grad[3][d] = -L * qB;
            grad[1][d] = c1A * qA + c1B * qB;
            grad[2][d] = c2A * qA + c2B * qB;
        }
    }
    return theta;
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
        double x[4][3], gdummy[4][3];
        for (int k = 0; k < 4; ++k) ld3(X, m.n, m.hinges[4 * i + k], x[k]);
        m.rest_theta[i] = hinge(x, gdummy, false);
    }
}

// Bending forces of every hinge on its four vertices: -k_b sin(theta - theta0) grad(theta).
__global__ void __launch_bounds__(256) k_mem_hinges(ib_membrane m, const double* X) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= m.nh) return;
    double x[4][3], gr[4][3];
    for (int k = 0; k < 4; ++k) ld3(X, m.n, m.hinges[4 * h + k], x[k]);
    const double th = hinge(x, gr, true);
    const double dE = m.k_bend * sin(th - m.rest_theta[h]);
    for (int k = 0; k < 4; ++k) {
        double* out = m.hinge_force + 3 * (int64_t)m.hinge_slot[4 * h + k];
        for (int d = 0; d < 3; ++d) out[d] = -dE * gr[k][d];
    }
}

// Inverse of the node -> hinge incidence CSR: position of (hinge, role) in hinge_inc.
__global__ void k_mem_hinge_slots(ib_membrane m, int64_t nnz) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) m.hinge_slot[m.hinge_inc[e]] = (int32_t)e;
}

// Per node: springs (CSR), the hinge forces of its incidences, tether.
__global__ void __launch_bounds__(256) k_mem_forces(ib_membrane m, const double* X, float* Fout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    double xi[3], xj[3], r[3], F[3] = {0.0, 0.0, 0.0};
    ld3(X, m.n, i, xi);
    if (m.nbr_ptr) {
        for (int e = m.nbr_ptr[i]; e < m.nbr_ptr[i + 1]; ++e) {
            ld3(X, m.n, m.nbr_idx[e], xj);
            sub(xj, xi, r);
            const double len = sqrt(dt3(r, r));
            const double s = m.k_spring * (len - m.rest_len[e]) / len;
            F[0] += s * r[0]; F[1] += s * r[1]; F[2] += s * r[2];
        }
    }
    if (m.hinge_ptr && m.k_bend != 0.0) {
        for (int e = m.hinge_ptr[i]; e < m.hinge_ptr[i + 1]; ++e) {
            const double* hf = m.hinge_force + 3 * (int64_t)e;
            F[0] += hf[0]; F[1] += hf[1]; F[2] += hf[2];
        }
    }
    if (m.anchors) {
        for (int d = 0; d < 3; ++d) F[d] -= m.k_tether * (xi[d] - m.anchors[d * m.n + i]);
    }
    for (int d = 0; d < 3; ++d) Fout[d * m.n + i] = (float)F[d];
}

hipError_t launch_membrane_rest(const ib_membrane* m, const double* X_rest, hipStream_t s) {
    const int64_t n = m->n > m->nh ? m->n : m->nh;
    if (n <= 0) return hipSuccess;
    k_mem_rest<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(*m, X_rest);
    if (m->hinge_ptr && m->nh > 0) {
        const int64_t nnz = 4 * m->nh;
        k_mem_hinge_slots<<<dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s>>>(*m, nnz);
    }
    return hipGetLastError();
}

hipError_t launch_membrane_forces(const ib_membrane* m, const double* X, float* F, hipStream_t s) {
    if (m->n <= 0) return hipSuccess;
    if (m->hinge_ptr && m->k_bend != 0.0 && m->nh > 0)
        k_mem_hinges<<<dim3((unsigned)((m->nh + 255) / 256)), dim3(256), 0, s>>>(*m, X);
    k_mem_forces<<<dim3((unsigned)((m->n + 255) / 256)), dim3(256), 0, s>>>(*m, X, F);
    return hipGetLastError();
}

}  // namespace lbmib
