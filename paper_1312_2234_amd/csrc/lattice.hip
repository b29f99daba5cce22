// lattice.hip -- lattice-Boltzmann kernels for gfx950 (section 3.3).
//
// State: weight-shifted populations g_i = f_i - w_i, in blocks of 64 consecutive cells
// ([ncell/64][19][64] per channel, see pidx), two buffers.  The stored buffer holds the post-collision values f* of the previous step
// ("pull" scheme), so one pass per step reads every population once from the neighbour
// it streams from and writes every population once, aligned, at its own cell:
//   152 B per cell per step in float32, 76 B in float16 / bfloat16.
// Work is split into 64-cell segments (one wavefront each) over all channels; a
// workgroup takes blockDim/64 consecutive segments.  With `remap` the workgroup order is
// permuted so that consecutive segments land on the same XCD (the dispatcher deals
// workgroups round-robin over the 8 XCDs), keeping the cache lines shared by adjacent
// segments (x-shifted loads straddle them) inside one L2.
#include "lbm_internal.h"

namespace lbmib {

// ---------------------------------------------------------------- one LBM step
// For every cell: pull (with bounce-back), moments (Eq. (17)-(18)), v = (j + F/2)/rho,
// shifted equilibrium of Eq. (20), Guo source of Eq. (19) (minus sign on the c_s^2 I
// term), BGK relaxation (Eq. (16)), aligned store into the other buffer.
template <class St, bool NT>
__global__ void __launch_bounds__(1024) k_step(LatArgs a) {
    using T = typename St::T;
    for_cells(a, [&](const Chan& ch, int32_t n) {
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        const int64_t N = ch.ncell;
        const T* s = (const T*)a.src + ch.pop_off;
        T* d = (T*)a.dst + ch.pop_off;
        float g[Q];
        pull<St>(s, ch, N, n, x, y, z, g);
        float drho, jx, jy, jz, Fx, Fy, Fz;
        moments(g, drho, jx, jy, jz);
        ib_force(a, ch, x, y, z, Fx, Fy, Fz);
        if (St::onsite && onsite_row(ch, y)) {
            onsite_wall(ch, y, g, Fx, Fy, Fz);
            moments(g, drho, jx, jy, jz);
        }
        const CellState cs = cell_state(drho, jx, jy, jz, Fx, Fy, Fz);
        const float om = ch.omega, guo = ch.guo;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float gn = bgk_c(i, g[i], cs, om, guo);
            if (NT)
                St::st_nt(d + pidx(i, n), gn);
            else
                St::st(d + pidx(i, n), gn);
        }
    });
}

// The same update for the cells of the flagged IB tiles only (TILE_PARTS workgroups per tile,
// one cell per thread), with their force.  Used after a full update with the body
// force alone: it overwrites exactly the cells whose IB force may be nonzero, with the
// values the fused update produces.  MERGE: a tile spread in several work items has only
// partial fixed-point blocks yet; this cell's sums are added here (as the merge kernel adds
// them) and the tile's force block is written for the later readers.
template <class St, bool MERGE>
__global__ void __launch_bounds__(TILE_CELLS) k_step_tiles(LatArgs a) {
    using T = typename St::T;
    const int nf = a.hdr->nflag;
    const int l = threadIdx.x + (int)(blockIdx.x % TILE_PARTS) * (TILE_CELLS / TILE_PARTS);
    for (int slot = blockIdx.x / TILE_PARTS; slot < nf; slot += gridDim.x / TILE_PARTS) {
        float f3[3];
        const int bigid = MERGE ? a.big[slot] : -1;
        if (MERGE && bigid >= 0) {
            const int nch = a.chunk_off[slot + 1] - a.chunk_off[slot];
            const unsigned long long* pb = a.part + (int64_t)bigid * (3 * TILE_CELLS) + l;
            unsigned long long v[3] = {0ull, 0ull, 0ull};
            for (int j = 0; j < nch; ++j)
#pragma unroll
                for (int k = 0; k < 3; ++k) v[k] += pb[(int64_t)j * (3 * TILE_CELLS) + k * TILE_CELLS];
            const bool nonfinite = a.hdr->nonfinite != 0;
            const double inv = ldexp(1.0, -a.hdr->scale_exp);
            float* fw = a.force_w + (int64_t)slot * (3 * TILE_CELLS) + l;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                f3[k] = nonfinite ? __builtin_nanf("") : (float)((double)(long long)v[k] * inv);
                fw[k * TILE_CELLS] = f3[k];
            }
        } else {
            const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS) + l;
#pragma unroll
            for (int k = 0; k < 3; ++k) f3[k] = fb[k * TILE_CELLS];
        }
        const Chan& ch = a.chan[a.flag_ch[slot]];
        const int t = (int)(a.flag_list[slot] - ch.tile_off);
        const int x = (t % ch.tnx) * TILE + (l & 7);
        const int y = ((t / ch.tnx) % ch.tny) * TILE + ((l >> 3) & 7);
        const int z = (t / (ch.tnx * ch.tny)) * TILE + (l >> 6);
        if (x >= ch.nx || y >= ch.ny || z >= ch.nz) continue;
        const int32_t n = x + ch.nx * (y + ch.ny * z);
        const T* s = (const T*)a.src + ch.pop_off;
        T* d = (T*)a.dst + ch.pop_off;
        float g[Q];
        pull<St>(s, ch, ch.ncell, n, x, y, z, g);
        float drho, jx, jy, jz, Fx, Fy, Fz;
        moments(g, drho, jx, jy, jz);
        // the body force plus this tile's IB force, as ib_force adds them
        Fx = ch.body[0];
        Fy = ch.body[1];
        Fz = ch.body[2];
        Fx += f3[0];
        Fy += f3[1];
        Fz += f3[2];
        if (St::onsite && onsite_row(ch, y)) {
            onsite_wall(ch, y, g, Fx, Fy, Fz);
            moments(g, drho, jx, jy, jz);
        }
        const CellState cs = cell_state(drho, jx, jy, jz, Fx, Fy, Fz);
        const float om = ch.omega, guo = ch.guo;
#pragma unroll
        for (int i = 0; i < Q; ++i) St::st(d + pidx(i, n), bgk_c(i, g[i], cs, om, guo));
    }
}

// Vector form of the same step: V consecutive cells of one x-row per lane (nx % V == 0,
// every channel a whole number of 64V-cell units), so every population is read and written
// with one aligned V-wide access per lane and a wavefront covers 64V consecutive cells of
// each of the 19 arrays.  Populations with c_x != 0 need the element just outside the
// lane's aligned group: it comes from the neighbouring lane by a lane shuffle, or by a
// direct load at a row end or at the edge of the wavefront.
template <class St, bool NT, int V>
__global__ void __launch_bounds__(256) k_step_v(LatArgs a) {
    using T = typename St::T;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t G = gridDim.x;
    int64_t L = a.remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    for (;; L += G) {
        const int64_t sw = (L * wpb + wave) * V;
        if (sw >= a.nseg) break;
        const int64_t seg = a.reverse ? a.nseg - V - sw : sw;  // nseg is a multiple of V
        const Chan& ch = a.chan[a.seg_ch[seg]];
        const int32_t n0 = (int32_t)((seg - ch.seg_off) * 64) + lane * V;
        int x0, y, z;
        cell_xyz(ch, (uint32_t)n0, x0, y, z);
        const int nx = ch.nx, ny = ch.ny, nz = ch.nz;
        const int32_t sxy = nx * ny;
        const int32_t oy_p = (y == 0) ? (ny - 1) * nx : -nx;
        const int32_t oy_m = (y == ny - 1) ? -(ny - 1) * nx : nx;
        const int32_t oz_p = (z == 0) ? (nz - 1) * sxy : -sxy;
        const int32_t oz_m = (z == nz - 1) ? -(nz - 1) * sxy : sxy;
        const bool wlo = ch.walls && y == 0;
        const bool whi = ch.walls && y == ny - 1;
        const int64_t N = ch.ncell;
        const T* s = (const T*)a.src + ch.pop_off;
        T* d = (T*)a.dst + ch.pop_off;
        const int32_t row0 = n0 - x0;
        float g[Q][V];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const bool bb = (cy(i) == 1 && wlo) || (cy(i) == -1 && whi);
            const int32_t row = row0 + (cy(i) == 1 ? oy_p : (cy(i) == -1 ? oy_m : 0)) +
                                (cz(i) == 1 ? oz_p : (cz(i) == -1 ? oz_m : 0));
            float A[V];
            ldv<St, V>(bb ? (s + pidx(opp(i), n0)) : (s + pidx(i, row + x0)), A);
            float corr = 0.0f;
            if (cy(i) != 0) {
                const float* u = cy(i) == 1 ? ch.uw_lo : ch.uw_hi;
                corr = bb ? 6.0f * wgt(i) * (cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2]) : 0.0f;
            }
            if (cx(i) == 1) {
                float prev = __shfl_up(A[V - 1], 1, 64);
                if (!bb && (x0 == 0 || lane == 0)) prev = St::ld(s + pidx(i, row + (x0 == 0 ? nx - 1 : x0 - 1)));
                g[i][0] = bb ? A[0] + corr : prev;
#pragma unroll
                for (int k = 1; k < V; ++k) g[i][k] = bb ? A[k] + corr : A[k - 1];
            } else if (cx(i) == -1) {
                float next = __shfl_down(A[0], 1, 64);
                if (!bb && (x0 + V == nx || lane == 63)) next = St::ld(s + pidx(i, row + (x0 + V == nx ? 0 : x0 + V)));
#pragma unroll
                for (int k = 0; k < V - 1; ++k) g[i][k] = bb ? A[k] + corr : A[k + 1];
                g[i][V - 1] = bb ? A[V - 1] + corr : next;
            } else {
#pragma unroll
                for (int k = 0; k < V; ++k) g[i][k] = A[k] + corr;
            }
        }
        // force: the V cells lie in one IB tile (V divides the tile edge)
        float Fx[V], Fy[V], Fz[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            Fx[k] = ch.body[0];
            Fy[k] = ch.body[1];
            Fz[k] = ch.body[2];
        }
        if (a.tile_slot) {
            const int slot = a.tile_slot[tile_of(ch, x0, y, z)];
            if (slot >= 0) {
                const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS) + tile_local(x0, y, z);
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    Fx[k] += fb[k];
                    Fy[k] += fb[TILE_CELLS + k];
                    Fz[k] += fb[2 * TILE_CELLS + k];
                }
            }
        }
        CellState cs[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            float gk[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) gk[i] = g[i][k];
            if (St::onsite && onsite_row(ch, y)) {
                onsite_wall(ch, y, gk, Fx[k], Fy[k], Fz[k]);
#pragma unroll
                for (int i = 0; i < Q; ++i) g[i][k] = gk[i];
            }
            float drho, jx, jy, jz;
            moments(gk, drho, jx, jy, jz);
            cs[k] = cell_state(drho, jx, jy, jz, Fx[k], Fy[k], Fz[k]);
        }
        const float om = ch.omega, guo = ch.guo;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float out[V];
#pragma unroll
            for (int k = 0; k < V; ++k) out[k] = bgk_c(i, g[i][k], cs[k], om, guo);
            stv<St, V, NT>(d + pidx(i, n0), out);
        }
        if (!a.persistent) break;
    }
}

// ---------------------------------------------------------------- initial state
// Un-stream: store s_i(x) such that the next pull yields the wanted pre-collision state
// h_i at every cell: s_i(x) = h_i(x + c_i), or h_opp(i)(x) + 6 w_i c_i.u_w when x + c_i
// is beyond a wall (the inverse of the bounce-back in `pull`).
template <class St, class Src>
__device__ __forceinline__ void unstream(const Chan& ch, typename St::T* d, int32_t n, int x, int y, int z,
                                         Src h) {
    const int64_t N = ch.ncell;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int32_t m;
        float v;
        if (step_out(ch, i, x, y, z, m))
            v = h(i, m);
        else
            v = h(opp(i), n) + wall_term(ch, i);
        St::st(d + pidx(i, n), v);
    }
}

template <class St>
__global__ void __launch_bounds__(1024) k_init(LatArgs a) {
    using T = typename St::T;
    for_cells(a, [&](const Chan& ch, int32_t n) {
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        T* d = (T*)a.dst + ch.pop_off;
        const int64_t N = ch.ncell;
        const float* rho = a.in_rho ? a.in_rho + ch.cell_off : nullptr;
        const float* u = a.in_u ? a.in_u + 3 * ch.cell_off : nullptr;
        auto h = [&](int i, int32_t m) {
            float dr = rho ? rho[m] - 1.0f : 0.0f;
            float ux, uy, uz;
            if (u) {
                ux = u[m];
                uy = u[N + m];
                uz = u[2 * N + m];
            } else if (ch.walls) {
                // steady wall-driven profile: walls at y = -1/2 and ny - 1/2, or on the rows
                // 0 and ny-1 (on-site walls)
                const int ym = (int)((m / ch.nx) % ch.ny);
                const float s = ch.walls == 2 ? (float)ym / (float)(ch.ny - 1) : ((float)ym + 0.5f) / (float)ch.ny;
                ux = ch.uw_lo[0] + (ch.uw_hi[0] - ch.uw_lo[0]) * s;
                uy = 0.0f;
                uz = ch.uw_lo[2] + (ch.uw_hi[2] - ch.uw_lo[2]) * s;
            } else {
                ux = uy = uz = 0.0f;
            }
            return geq_i(i, dr, ux, uy, uz);
        };
        unstream<St>(ch, d, n, x, y, z, h);
    });
}

template <class St>
__global__ void __launch_bounds__(1024) k_setf(LatArgs a) {
    using T = typename St::T;
    for_cells(a, [&](const Chan& ch, int32_t n) {
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        T* d = (T*)a.dst + ch.pop_off;
        const int64_t N = ch.ncell;
        const float* f = a.in_f + (int64_t)Q * ch.cell_off;
        auto h = [&](int i, int32_t m) { return f[(int64_t)i * N + m] - wgt(i); };
        unstream<St>(ch, d, n, x, y, z, h);
    });
}

// ---------------------------------------------------------------- read-outs
template <class St>
__global__ void __launch_bounds__(1024) k_moments(LatArgs a) {
    using T = typename St::T;
    for_cells(a, [&](const Chan& ch, int32_t n) {
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        const int64_t N = ch.ncell;
        float g[Q];
        pull<St>((const T*)a.src + ch.pop_off, ch, N, n, x, y, z, g);
        float drho, jx, jy, jz, Fx, Fy, Fz;
        ib_force(a, ch, x, y, z, Fx, Fy, Fz);
        if (St::onsite && onsite_row(ch, y)) onsite_wall(ch, y, g, Fx, Fy, Fz);
        moments(g, drho, jx, jy, jz);
        const float ir = 1.0f / (1.0f + drho);
        if (a.out_rho) a.out_rho[ch.cell_off + n] = drho;
        if (a.out_v) {
            float* v = a.out_v + 3 * ch.cell_off;
            v[n] = (jx + 0.5f * Fx) * ir;
            v[N + n] = (jy + 0.5f * Fy) * ir;
            v[2 * N + n] = (jz + 0.5f * Fz) * ir;
        }
    });
}

template <class St>
__global__ void __launch_bounds__(1024) k_getf(LatArgs a) {
    using T = typename St::T;
    for_cells(a, [&](const Chan& ch, int32_t n) {
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        const int64_t N = ch.ncell;
        float g[Q];
        pull<St>((const T*)a.src + ch.pop_off, ch, N, n, x, y, z, g);
        if (St::onsite && onsite_row(ch, y)) {
            float Fx, Fy, Fz;
            ib_force(a, ch, x, y, z, Fx, Fy, Fz);
            onsite_wall(ch, y, g, Fx, Fy, Fz);
        }
        float* f = a.out_f + (int64_t)Q * ch.cell_off;
#pragma unroll
        for (int i = 0; i < Q; ++i) f[(int64_t)i * N + n] = g[i] + wgt(i);
    });
}

// Wall stress at rows y = 0 and y = ny-1, one thread per (x, z, side).  Output index
// space: per channel [2 sides][nx*nz], channels concatenated (Chan::wss_off).
template <class St>
__global__ void __launch_bounds__(256) k_wss(LatArgs a, int nch, int64_t total) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    using T = typename St::T;
    if (gid >= total) return;
    int c = 0;  // channel owning this output element (few channels: linear search)
    while (c + 1 < nch && gid >= a.chan[c + 1].wss_off) ++c;
    const Chan& ch = a.chan[c];
    const int64_t k = gid - ch.wss_off;
    const int64_t plane = (int64_t)ch.nx * ch.nz;
    const int side = k >= plane ? 1 : 0;
    const int64_t q = k - side * plane;
    const int x = (int)(q % ch.nx), z = (int)(q / ch.nx);
    const int y = side ? ch.ny - 1 : 0;
    const int32_t n = x + ch.nx * (y + ch.ny * z);
    const int64_t N = ch.ncell;
    float g[Q];
    pull<St>((const T*)a.src + ch.pop_off, ch, N, n, x, y, z, g);
    float drho, jx, jy, jz, Fx, Fy, Fz;
    ib_force(a, ch, x, y, z, Fx, Fy, Fz);
    if (St::onsite && onsite_row(ch, y)) onsite_wall(ch, y, g, Fx, Fy, Fz);
    moments(g, drho, jx, jy, jz);
    const float rho = 1.0f + drho, ir = 1.0f / rho;
    const float vx = (jx + 0.5f * Fx) * ir, vy = (jy + 0.5f * Fy) * ir, vz = (jz + 0.5f * Fz) * ir;
    float sxy = 0.f, szy = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cy(i) == 0) continue;
        const float neq = g[i] - geq_i(i, drho, vx, vy, vz);
        if (cx(i)) sxy += (float)(cx(i) * cy(i)) * neq;
        if (cz(i)) szy += (float)(cz(i) * cy(i)) * neq;
    }
    const float k2 = 1.0f - 0.5f * ch.omega;
    float* out = (side ? a.out_hi : a.out_lo) + ch.wss_off;
    out[q] = -k2 * sxy - k2 * 0.5f * (Fx * vy + Fy * vx);
    out[plane + q] = -k2 * szy - k2 * 0.5f * (Fz * vy + Fy * vz);
}

// STREAM-style copy used to measure the practical HBM ceiling (16 bytes per lane per
// iteration, grid-stride; variant 1 stores non-temporally).
typedef float f4v __attribute__((ext_vector_type(4)));
template <bool NT>
__global__ void __launch_bounds__(256) k_copy16(const f4v* __restrict__ src, f4v* __restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const f4v v = src[i];
        if (NT)
            __builtin_nontemporal_store(v, dst + i);
        else
            dst[i] = v;
    }
}

hipError_t launch_copy16(hipStream_t s, const void* src, void* dst, int64_t bytes, int variant, int64_t grid) {
    const int64_t n16 = bytes / 16;
    if (grid <= 0) grid = (n16 + 255) / 256;
    if (variant == 1)
        k_copy16<true><<<dim3((unsigned)grid), dim3(256), 0, s>>>((const f4v*)src, (f4v*)dst, n16);
    else
        k_copy16<false><<<dim3((unsigned)grid), dim3(256), 0, s>>>((const f4v*)src, (f4v*)dst, n16);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_fill_i32<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, n, v);
    return hipGetLastError();
}

template <class St, int V>
static hipError_t launch_step_v(lbm_ctx* c, const LatArgs& a0) {
    LatArgs a = a0;
    const int block = 256, wpb = 4;
    const int64_t units = c->total_segs / V;
    const int64_t nblk = (units + wpb - 1) / wpb;
    int64_t grid = nblk;
    a.remap = c->launch.xcd_remap;
    a.persistent = 0;
    if (c->launch.persistent > 0 && c->launch.persistent < nblk) {
        grid = c->launch.persistent;
        a.persistent = 1;
    }
    if (c->launch.nontemporal)
        k_step_v<St, true, V><<<dim3((unsigned)grid), dim3(block), 0, c->stream>>>(a);
    else
        k_step_v<St, false, V><<<dim3((unsigned)grid), dim3(block), 0, c->stream>>>(a);
    return hipGetLastError();
}

// The vector step applies when every channel has nx % V == 0 and a whole number of
// 64V-cell units; otherwise the scalar step runs.
static bool vec_ok(const lbm_ctx* c, int V) {
    for (const Chan& ch : c->chans)
        if (ch.nx % V != 0 || ch.ncell % (64 * V) != 0) return false;
    return true;
}

template <class St>
static hipError_t launch_typed(lbm_ctx* c, int which, const LatArgs& a0) {
    if (which == LK_STEP && c->launch.vec == 4 && vec_ok(c, 4)) return launch_step_v<St, 4>(c, a0);
    if (which == LK_STEP && c->launch.vec == 2 && vec_ok(c, 2)) return launch_step_v<St, 2>(c, a0);
    LatArgs a = a0;
    const int block = c->launch.block;
    const int wpb = block / 64;
    const int64_t nblk = (c->total_segs + wpb - 1) / wpb;
    int64_t grid = nblk;
    a.remap = c->launch.xcd_remap;
    a.persistent = 0;
    if (which == LK_STEP && c->launch.persistent > 0 && c->launch.persistent < nblk) {
        grid = c->launch.persistent;
        a.persistent = 1;
    }
    if (which != LK_STEP) a.remap = 0;
    dim3 g((unsigned)grid), b((unsigned)block);
    switch (which) {
        case LK_STEP:
            if (c->launch.nontemporal)
                k_step<St, true><<<g, b, 0, c->stream>>>(a);
            else
                k_step<St, false><<<g, b, 0, c->stream>>>(a);
            break;
        case LK_INIT: k_init<St><<<g, b, 0, c->stream>>>(a); break;
        case LK_MOMENTS: k_moments<St><<<g, b, 0, c->stream>>>(a); break;
        case LK_GETF: k_getf<St><<<g, b, 0, c->stream>>>(a); break;
        case LK_SETF: k_setf<St><<<g, b, 0, c->stream>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class St>
static hipError_t launch_wss_typed(lbm_ctx* c, const LatArgs& a, int64_t total) {
    const int64_t blocks = (total + 255) / 256;
    k_wss<St><<<dim3((unsigned)blocks), dim3(256), 0, c->stream>>>(a, c->nch, total);
    return hipGetLastError();
}

hipError_t launch_lattice(lbm_ctx* c, int which, const LatArgs& a) {
    return with_storage(c, [&](auto st) { return launch_typed<decltype(st)>(c, which, a); });
}

template <class St>
static void launch_tiles_typed(lbm_ctx* c, const LatArgs& a, bool merge, dim3 grid, dim3 block) {
    if (merge)
        k_step_tiles<St, true><<<grid, block, 0, c->stream>>>(a);
    else
        k_step_tiles<St, false><<<grid, block, 0, c->stream>>>(a);
}

hipError_t launch_step_tiles(lbm_ctx* c, const LatArgs& a, bool merge) {
    int64_t g = c->max_slots < c->ib_grid ? c->max_slots : c->ib_grid;
    if (g < 1) g = 1;
    const dim3 grid((unsigned)(g * TILE_PARTS)), block(TILE_CELLS / TILE_PARTS);
    with_storage(c, [&](auto st) { launch_tiles_typed<decltype(st)>(c, a, merge, grid, block); });
    return hipGetLastError();
}

hipError_t launch_wss(lbm_ctx* c, const LatArgs& a, int64_t total) {
    return with_storage(c, [&](auto st) { return launch_wss_typed<decltype(st)>(c, a, total); });
}

}  // namespace lbmib
