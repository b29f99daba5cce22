// lbm_device.h -- device-side building blocks shared by the library's kernels.
//
// D3Q19 in the paper's numbering (section 3.3, Eq. (21); the order of the directions
// is the one fixed by the on-site wall equations Eq. (23)-(30)), population storage
// codecs for the weight-shifted state g_i = f_i - w_i, the per-channel descriptor and
// the pull-streaming gather with halfway bounce-back at the y-walls.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmib {

constexpr int Q = 19;
constexpr int TILE = 8;               // immersed-boundary tile edge (cells)
constexpr int TILE_CELLS = TILE * TILE * TILE;

__host__ __device__ constexpr int cx(int i) {
    constexpr int t[Q] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int t[Q] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
    return t[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int t[Q] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
    return t[i];
}
__host__ __device__ constexpr int opp(int i) {
    constexpr int t[Q] = {1, 0, 3, 2, 5, 4, 11, 10, 13, 12, 7, 6, 9, 8, 17, 16, 15, 14, 18};
    return t[i];
}
__host__ __device__ constexpr float wgt(int i) {
    return i < 6 ? 1.0f / 18.0f : (i < 18 ? 1.0f / 36.0f : 1.0f / 3.0f);
}

// Per-channel descriptor (device copy in the workspace; read with scalar loads).
struct Chan {
    int32_t nx, ny, nz, walls;
    int64_t ncell;     // nx*ny*nz (< 2^31)
    int64_t pop_off;   // element offset of this channel's [ncell/64][19][64] population blocks
    int64_t cell_off;  // offset of this channel in concatenated per-cell outputs
    int64_t seg_off;   // first 64-cell segment of this channel
    int64_t tile_off;  // first IB tile of this channel
    int64_t node_lo, node_hi;  // immersed-boundary nodes of this channel
    int64_t wss_off;   // offset in the concatenated [2][nz][nx] wall-stress outputs
    int32_t tnx, tny, tnz, pad0;  // IB tiles per axis
    uint32_t mx, sx, my, sy;      // fast division by nx and ny
    float tau, omega, guo, pad1;  // tau, 1/tau, 1 - 1/(2 tau)
    float body[3];
    float uw_lo[3];
    float uw_hi[3];
    float pad2[3];
};

// Population layout: blocks of 64 consecutive cells (one wavefront's segment), each block
// holding its 19 populations one after another ([cells/64][19][64], "AoSoA").  A wavefront
// then writes one contiguous 19 x 64-element run per step and reads 64-element runs,
// instead of touching 19 + 19 arrays a whole lattice apart.
constexpr int BLK = 64;
__device__ __forceinline__ int64_t pidx(int i, int32_t n) {
    return (int64_t)(n >> 6) * (Q * BLK) + i * BLK + (n & (BLK - 1));
}

// q = n / d for n < 2^31 (round-up reciprocal, see host set-up).
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m, uint32_t s) {
    return (__umulhi(n, m) + n) >> s;
}

__device__ __forceinline__ void cell_xyz(const Chan& ch, uint32_t n, int& x, int& y, int& z) {
    uint32_t q = fdiv(n, ch.mx, ch.sx);
    x = (int)(n - q * (uint32_t)ch.nx);
    uint32_t r = fdiv(q, ch.my, ch.sy);
    y = (int)(q - r * (uint32_t)ch.ny);
    z = (int)r;
}

// ---------------------------------------------------------------- storage codecs
struct StF32 {
    static constexpr bool onsite = false;  // no channel with on-site walls
    using T = float;
    static __device__ __forceinline__ float dec(T v) { return v; }
    static __device__ __forceinline__ T enc(float v) { return v; }
    static __device__ __forceinline__ float ld(const T* p) { return *p; }
    static __device__ __forceinline__ void st(T* p, float v) { *p = v; }
    static __device__ __forceinline__ void st_nt(T* p, float v) { __builtin_nontemporal_store(v, p); }
};
struct StF16 {
    static constexpr bool onsite = false;  // no channel with on-site walls
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v) { return __half2float(__ushort_as_half(v)); }
    static __device__ __forceinline__ float ld(const T* p) { return dec(*p); }
    static __device__ __forceinline__ uint16_t enc(float v) { return __half_as_ushort(__float2half_rn(v)); }
    static __device__ __forceinline__ void st(T* p, float v) { *p = enc(v); }
    static __device__ __forceinline__ void st_nt(T* p, float v) { __builtin_nontemporal_store(enc(v), p); }
};
struct StBF16 {
    static constexpr bool onsite = false;  // no channel with on-site walls
    using T = uint16_t;
    static __device__ __forceinline__ float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
    static __device__ __forceinline__ float ld(const T* p) { return dec(*p); }
    // round to nearest, ties to even, NaN stays NaN: the hardware conversion (one
    // v_cvt_pk_bf16_f32), equal on every float32 input to the integer rounding
    // u + 0x7fff + (u >> 16 & 1) taken >> 16
    static __device__ __forceinline__ uint16_t enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    static __device__ __forceinline__ void st(T* p, float v) { *p = enc(v); }
    static __device__ __forceinline__ void st_nt(T* p, float v) { __builtin_nontemporal_store(enc(v), p); }
};

// The same storage form for a context with at least one on-site-wall channel: the kernels
// compile their wall-row branch only for these, so the others keep the plain code.
template <class Base>
struct OnSite : Base {
    static constexpr bool onsite = true;
};

// V consecutive stored elements (address aligned to V elements) <-> floats.
template <class St, int V>
__device__ __forceinline__ void ldv(const typename St::T* p, float out[V]) {
    using T = typename St::T;
    typedef T vec __attribute__((ext_vector_type(V)));
    const vec t = *(const vec*)p;
#pragma unroll
    for (int k = 0; k < V; ++k) out[k] = St::dec(t[k]);
}
template <class St, int V, bool NT>
__device__ __forceinline__ void stv(typename St::T* p, const float in[V]) {
    using T = typename St::T;
    typedef T vec __attribute__((ext_vector_type(V)));
    vec t;
#pragma unroll
    for (int k = 0; k < V; ++k) t[k] = St::enc(in[k]);
    if (NT)
        __builtin_nontemporal_store(t, (vec*)p);
    else
        *(vec*)p = t;
}

// ---------------------------------------------------------------- pull streaming
// Populations arriving at cell n = (x, y, z) of the current step: f_i(x) = f*_i(x - c_i)
// with x, z periodic; when x - c_i lies beyond a y-wall the halfway bounce-back gives
// f_i(x) = f*_opp(i)(x) + 6 w_i c_i.u_w.  In the shifted variables the same relation
// holds for g = f - w because w_i = w_opp(i).  `s` points at the channel's block.  With
// on-site walls the entering populations of a wall row are loaded the same way and then
// replaced by onsite_wall().  pull = pull_loads (the stored values, the bounce-back source
// chosen) then pull_walls (the moving-wall term), which a kernel may also call apart, with
// the loads issued ahead of their use.
template <class St>
__device__ __forceinline__ void pull_loads(const typename St::T* __restrict__ s, const Chan& ch, int32_t n, int x,
                                           int y, int z, float g[Q]) {
    const int nx = ch.nx, ny = ch.ny, nz = ch.nz;
    const int32_t sxy = nx * ny;
    const int32_t ox_p = (x == 0) ? (nx - 1) : -1;          // c_x = +1 comes from x-1
    const int32_t ox_m = (x == nx - 1) ? -(nx - 1) : 1;     // c_x = -1 comes from x+1
    const int32_t oy_p = (y == 0) ? (ny - 1) * nx : -nx;
    const int32_t oy_m = (y == ny - 1) ? -(ny - 1) * nx : nx;
    const int32_t oz_p = (z == 0) ? (nz - 1) * sxy : -sxy;
    const int32_t oz_m = (z == nz - 1) ? -(nz - 1) * sxy : sxy;
    const bool wlo = ch.walls && y == 0;
    const bool whi = ch.walls && y == ny - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int32_t off = (cx(i) == 1 ? ox_p : (cx(i) == -1 ? ox_m : 0)) +
                      (cy(i) == 1 ? oy_p : (cy(i) == -1 ? oy_m : 0)) +
                      (cz(i) == 1 ? oz_p : (cz(i) == -1 ? oz_m : 0));
        const bool bb = (cy(i) == 1 && wlo) || (cy(i) == -1 && whi);
        const typename St::T* p = bb ? (s + pidx(opp(i), n)) : (s + pidx(i, n + off));
        g[i] = St::ld(p);
    }
}

// The moving-wall term of the bounced-back populations, added to the loaded values.
__device__ __forceinline__ void pull_walls(const Chan& ch, int y, float g[Q]) {
    const bool wlo = ch.walls && y == 0;
    const bool whi = ch.walls && y == ch.ny - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (cy(i) != 0) {
            const bool bb = (cy(i) == 1 && wlo) || (cy(i) == -1 && whi);
            const float* u = cy(i) == 1 ? ch.uw_lo : ch.uw_hi;
            float corr = 6.0f * wgt(i) * (cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2]);
            g[i] += bb ? corr : 0.0f;
        }
}

template <class St>
__device__ __forceinline__ void pull(const typename St::T* __restrict__ s, const Chan& ch, int64_t N,
                                     int32_t n, int x, int y, int z, float g[Q]) {
    pull_loads<St>(s, ch, n, x, y, z, g);
    pull_walls(ch, y, g);
}

// On-site velocity walls (Chan::walls == 2; Eq. (23)-(30), turned to a y-normal wall).  The
// walls lie on the rows y = 0 and y = ny-1; there the populations entering the fluid
// (c.n = +1 for the inward normal n = +y on row 0, -y on row ny-1) have no source cell and
// are set from the others so that the cell's velocity (sum c f + F/2)/rho is the wall's.
// With J = rho u_w - F/2 (F the cell's force):
//   rho (1 - n.u_w) = sum_{c.n=0} f + 2 sum_{c.n=-1} f - n.F/2
//   N_t = sum_{c.n=0} c_t f / 2 - J_t / 3          (t = x, z)
//   f_i = f_opp(i) + 6 w_i c_i.J - sum_t c_it N_t   (c_i.n = +1)
// In the shifted variables g = f - w the weights drop out: those of c.n = 0 plus twice those
// of c.n = -1 sum to 1, the c.n = 0 ones are symmetric in c_t, and w_i = w_opp(i); so
// rho - 1 = (S_0 + 2 S_- - n.F/2 + n.u_w) / (1 - n.u_w) over the shifted sums S.
//
// The kernels compile the wall-row branch only for the OnSite<> storage forms (contexts
// with an on-site-wall channel), take the moments of the pull first, so that the loads of
// the cell's force overlap them, and on a wall row apply the rule and take the moments again.

// True on the wall rows of a channel with on-site walls.
__device__ __forceinline__ bool onsite_row(const Chan& ch, int y) {
    return ch.walls == 2 && (y == 0 || y == ch.ny - 1);
}

// Applies the on-site rule to a pulled cell of a wall row (onsite_row true).  One body serves both walls:
// every array index is a compile-time constant and the wall only selects values (two
// inlined copies chosen at run time get merged by the compiler into stores at a selected
// index, which moves the array to scratch memory).
__device__ __forceinline__ void onsite_wall(const Chan& ch, int y, float g[Q], float Fx, float Fy, float Fz) {
    const bool lo = y == 0;  // inward normal +y on row 0, -y on row ny-1
    const float sn = lo ? 1.0f : -1.0f;
    const float ux = lo ? ch.uw_lo[0] : ch.uw_hi[0];
    const float uy = lo ? ch.uw_lo[1] : ch.uw_hi[1];
    const float uz = lo ? ch.uw_lo[2] : ch.uw_hi[2];
    float s0 = 0.f, sm = 0.f, px = 0.f, pz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cy(i) == 0) {
            s0 += g[i];
            if (cx(i)) px += cx(i) * g[i];
            if (cz(i)) pz += cz(i) * g[i];
        } else {
            sm += ((cy(i) == 1) != lo) ? g[i] : 0.0f;  // leaving through the wall: c.n = -1
        }
    }
    const float un = sn * uy;
    const float drho = (s0 + 2.0f * sm - 0.5f * sn * Fy + un) / (1.0f - un);
    const float rho = 1.0f + drho;
    const float Jx = rho * ux - 0.5f * Fx, Jy = rho * uy - 0.5f * Fy, Jz = rho * uz - 0.5f * Fz;
    const float Nx = 0.5f * px - Jx * (1.0f / 3.0f), Nz = 0.5f * pz - Jz * (1.0f / 3.0f);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (cy(i) != 0) {
            const float v = g[opp(i)] + 6.0f * wgt(i) * (cx(i) * Jx + cy(i) * Jy + cz(i) * Jz) - (cx(i) * Nx + cz(i) * Nz);
            g[i] = ((cy(i) == 1) == lo) ? v : g[i];  // entering the fluid: c.n = +1
        }
}

// Zeroth and first moments of the shifted populations: drho = sum g, j = sum c g
// (Eq. (17)-(18) with sum w = 1 and sum w c = 0).
__device__ __forceinline__ void moments(const float g[Q], float& drho, float& jx, float& jy, float& jz) {
    float r = 0.f, a = 0.f, b = 0.f, c = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r += g[i];
        if (cx(i)) a += cx(i) * g[i];
        if (cy(i)) b += cy(i) * g[i];
        if (cz(i)) c += cz(i) * g[i];
    }
    drho = r; jx = a; jy = b; jz = c;
}

// Shifted equilibrium of Eq. (20) at rho = 1 + drho and velocity u.
__device__ __forceinline__ float geq_i(int i, float drho, float ux, float uy, float uz) {
    const float rho = 1.0f + drho;
    const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    return wgt(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * (ux * ux + uy * uy + uz * uz)));
}

// Cell reached from (x,y,z) along +c_i (x, z periodic; y periodic only without walls).
// Returns false if +c_i leaves through a wall.
__device__ __forceinline__ bool step_out(const Chan& ch, int i, int x, int y, int z, int32_t& m) {
    int xs = x + cx(i), ys = y + cy(i), zs = z + cz(i);
    if (ys < 0 || ys >= ch.ny) {
        if (ch.walls) return false;
        ys = ys < 0 ? ys + ch.ny : ys - ch.ny;
    }
    xs = xs < 0 ? xs + ch.nx : (xs >= ch.nx ? xs - ch.nx : xs);
    zs = zs < 0 ? zs + ch.nz : (zs >= ch.nz ? zs - ch.nz : zs);
    m = xs + ch.nx * (ys + ch.ny * zs);
    return true;
}

__device__ __forceinline__ float wall_term(const Chan& ch, int i) {
    // population i leaving through the wall on its own side: c_iy = +1 -> upper, -1 -> lower
    const float* u = cy(i) > 0 ? ch.uw_hi : ch.uw_lo;
    return 6.0f * wgt(i) * (cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2]);
}

// ---------------------------------------------------------------- forced BGK collision
// Eq. (16) with the equilibrium of Eq. (20) and the Guo source of Eq. (19) (minus sign on
// the c_s^2 I term), in shifted variables.  Every rounding is fixed here (explicit fused
// multiply-adds, no contraction left to the compiler), so that each kernel applying the
// collision -- the plain step, its vector form and the closure step -- gives the same bits.
struct CellState {
    float drho, rho, vx, vy, vz, Fx, Fy, Fz, vv15, vF3;
};

// v = (j + F/2) / rho, 1.5 v.v and 3 v.F
__device__ __forceinline__ CellState cell_state(float drho, float jx, float jy, float jz, float Fx, float Fy,
                                                float Fz) {
#pragma clang fp contract(off)
    CellState s;
    s.drho = drho;
    s.rho = 1.0f + drho;
    const float ir = 1.0f / s.rho;
    s.vx = fmaf(0.5f, Fx, jx) * ir;
    s.vy = fmaf(0.5f, Fy, jy) * ir;
    s.vz = fmaf(0.5f, Fz, jz) * ir;
    s.Fx = Fx;
    s.Fy = Fy;
    s.Fz = Fz;
    s.vv15 = 1.5f * fmaf(s.vx, s.vx, fmaf(s.vy, s.vy, s.vz * s.vz));
    s.vF3 = 3.0f * fmaf(s.vx, Fx, fmaf(s.vy, Fy, s.vz * Fz));
    return s;
}

// c_i . (x, y, z) for the compile-time direction i (additions only)
__device__ __forceinline__ float cdot(int i, float x, float y, float z) {
#pragma clang fp contract(off)
    float r = 0.0f;
    bool any = false;
    if (cx(i) != 0) { r = cx(i) > 0 ? x : -x; any = true; }
    if (cy(i) != 0) { r = any ? (cy(i) > 0 ? r + y : r - y) : (cy(i) > 0 ? y : -y); any = true; }
    if (cz(i) != 0) { r = any ? (cz(i) > 0 ? r + z : r - z) : (cz(i) > 0 ? z : -z); any = true; }
    return r;
}

// shifted equilibrium w_i (drho + rho (3 c.v + 4.5 (c.v)^2 - 1.5 v.v))
__device__ __forceinline__ float geq_c(int i, const CellState& s) {
#pragma clang fp contract(off)
    const float cu = cdot(i, s.vx, s.vy, s.vz);
    return wgt(i) * fmaf(s.rho, fmaf(fmaf(4.5f, cu, 3.0f), cu, -s.vv15), s.drho);
}

// post-collision shifted population g - (g - geq)/tau + S_i
__device__ __forceinline__ float bgk_c(int i, float g, const CellState& s, float om, float guo) {
#pragma clang fp contract(off)
    const float cu = cdot(i, s.vx, s.vy, s.vz);
    const float cF = cdot(i, s.Fx, s.Fy, s.Fz);
    const float geq = geq_c(i, s);
    const float S = (wgt(i) * guo) * fmaf(fmaf(9.0f, cu, 3.0f), cF, -s.vF3);
    return fmaf(-om, g - geq, g) + S;
}

// The same with g - geq already at hand (the same bits as bgk_c)
__device__ __forceinline__ float bgk_from_neq(int i, float g, float neq, const CellState& s, float om, float guo) {
#pragma clang fp contract(off)
    const float cu = cdot(i, s.vx, s.vy, s.vz);
    const float cF = cdot(i, s.Fx, s.Fy, s.Fz);
    const float S = (wgt(i) * guo) * fmaf(fmaf(9.0f, cu, 3.0f), cF, -s.vF3);
    return fmaf(-om, neq, g) + S;
}

// IB force-field lookup: tile of the cell -> slot (or -1) -> [3][512] block.
__device__ __forceinline__ int64_t tile_of(const Chan& ch, int x, int y, int z) {
    return ch.tile_off + (x >> 3) + (int64_t)ch.tnx * ((y >> 3) + (int64_t)ch.tny * (z >> 3));
}
__device__ __forceinline__ int tile_local(int x, int y, int z) {
    return ((z & 7) << 6) | ((y & 7) << 3) | (x & 7);
}

}  // namespace lbmib
