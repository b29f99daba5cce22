// closure.hip -- learned collision closure on the gfx950 BF16 matrix cores.
//
// The paper's collision is the forced BGK update of Eq. (16) with the source of Eq. (19)
// and the equilibrium of Eq. (20).  This file adds a learned correction of the
// non-conserved moments of that update (not in the paper):
//
//   m   = M_nc (g - g^eq)                 15 non-equilibrium moments, pre-collision
//   x   = ((m, |F_IB|) - mean) * scale    16 network inputs (BF16)
//   y   = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3     16 -> 64 -> 64 -> 16
//   dm  = y[0:15] * out_scale
//   g*  = g*_BGK + M_nc^T dm              only if dm is finite and |dm| <= c |m|
//
// M is the orthonormal D3Q19 moment basis obtained by Gram-Schmidt of the monomials
// 1, x, y, z, x^2, y^2, z^2, xy, xz, yz, x^2y, x^2z, y^2x, y^2z, z^2x, z^2y, x^2y^2,
// x^2z^2, y^2z^2 of the lattice velocities, computed here at compile time; rows 4..18
// (M_nc) are orthogonal to 1 and c, so the correction leaves mass and momentum unchanged.
//
// Matrix-core mapping (v_mfma_f32_16x16x16_bf16): a wavefront holds 64 cells, one per
// lane.  Layers are evaluated transposed, H^T = W^T X^T, with the weights as the A operand
// and the activations as the B operand: the accumulator layout of one layer (row
// 4*(lane/16)+r, column lane%16) is then exactly the B-operand layout of the next, so
// activations never leave registers.  The cell-per-lane features enter through a
// 2 KB LDS transpose and the outputs leave through a 4 KB one.
//
// Training uses the same forward pass and the transposed chain rule on the matrix cores;
// weight gradients contract over cells through LDS-transposed activation tiles; partial
// gradients of every workgroup are reduced in a fixed order (bitwise reproducible).
#include "lbm_internal.h"

namespace lbmib {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float acc4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- moment basis
constexpr double c_sqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int it = 0; it < 200; ++it) r = 0.5 * (r + x / r);
    return r;
}

struct Basis {
    float m[MLP_NNC][Q];  // non-conserved rows 4..18
};

constexpr Basis make_basis() {
    constexpr int ex[Q][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
                              {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1},
                              {1, 0, 2}, {0, 1, 2}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
    double rows[Q][Q] = {};
    for (int k = 0; k < Q; ++k) {
        double v[Q] = {};
        for (int i = 0; i < Q; ++i) {
            double p = 1.0;
            for (int e = 0; e < ex[k][0]; ++e) p *= cx(i);
            for (int e = 0; e < ex[k][1]; ++e) p *= cy(i);
            for (int e = 0; e < ex[k][2]; ++e) p *= cz(i);
            v[i] = p;
        }
        for (int pass = 0; pass < 2; ++pass)
            for (int r = 0; r < k; ++r) {
                double d = 0.0;
                for (int i = 0; i < Q; ++i) d += rows[r][i] * v[i];
                for (int i = 0; i < Q; ++i) v[i] -= d * rows[r][i];
            }
        double nn = 0.0;
        for (int i = 0; i < Q; ++i) nn += v[i] * v[i];
        const double inv = 1.0 / c_sqrt(nn);
        for (int i = 0; i < Q; ++i) rows[k][i] = v[i] * inv;
    }
    Basis b{};
    for (int k = 0; k < MLP_NNC; ++k)
        for (int i = 0; i < Q; ++i) {
            const double x = rows[k + 4][i];
            b.m[k][i] = (x < 1e-12 && x > -1e-12) ? 0.0f : (float)x;
        }
    return b;
}

constexpr Basis kBasis = make_basis();

// Opposite velocities come in 9 pairs (i, opp(i)), plus the rest velocity.  Gram-Schmidt
// only mixes monomials of equal degree parity (a product of odd and even components sums
// to zero over the velocity set), so every row of the basis is even (M[k][opp i] = M[k][i])
// or odd (M[k][opp i] = -M[k][i]): an even moment needs only the pair sums, an odd one only
// the differences, which halves both transforms.
constexpr int kPairs = 9;
constexpr int kPairLo[kPairs] = {0, 2, 4, 6, 7, 8, 9, 14, 15};

constexpr int row_parity(int k) {  // 0 even, 1 odd, -1 neither
    bool even = true, odd = true;
    for (int i = 0; i < Q; ++i) {
        even = even && kBasis.m[k][opp(i)] == kBasis.m[k][i];
        odd = odd && kBasis.m[k][opp(i)] == -kBasis.m[k][i];
    }
    return even ? 0 : (odd ? 1 : -1);
}
constexpr bool pairs_ok() {
    for (int p = 0; p < kPairs; ++p)
        if (opp(kPairLo[p]) <= kPairLo[p]) return false;
    for (int k = 0; k < MLP_NNC; ++k) {
        if (row_parity(k) < 0) return false;
        if (row_parity(k) == 1 && kBasis.m[k][Q - 1] != 0.0f) return false;
    }
    return opp(Q - 1) == Q - 1;
}
static_assert(pairs_ok(), "moment basis rows must have a definite parity");

// m_k = sum_i M_nc[k][i] d_i; zero entries of the basis are skipped at compile time.
__device__ __forceinline__ void to_moments(const float d[Q], float m[MLP_NNC]) {
    float sp[kPairs], dp[kPairs];
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        sp[p] = d[kPairLo[p]] + d[opp(kPairLo[p])];
        dp[p] = d[kPairLo[p]] - d[opp(kPairLo[p])];
    }
#pragma unroll
    for (int k = 0; k < MLP_NNC; ++k) {
        const bool odd = row_parity(k) == 1;
        float s = 0.0f;
#pragma unroll
        for (int p = 0; p < kPairs; ++p)
            if (kBasis.m[k][kPairLo[p]] != 0.0f) s += kBasis.m[k][kPairLo[p]] * (odd ? dp[p] : sp[p]);
        if (!odd && kBasis.m[k][Q - 1] != 0.0f) s += kBasis.m[k][Q - 1] * d[Q - 1];
        m[k] = s;
    }
}

// d_i = sum_k M_nc[k][i] m_k for every i: per pair, the even rows' sum E and the odd rows'
// sum O give d_i = E + O and d_opp(i) = E - O.
__device__ __forceinline__ void from_moments(const float m[MLP_NNC], float d[Q]) {
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const int i = kPairLo[p];
        float e = 0.0f, o = 0.0f;
#pragma unroll
        for (int k = 0; k < MLP_NNC; ++k)
            if (kBasis.m[k][i] != 0.0f) {
                if (row_parity(k) == 1)
                    o += kBasis.m[k][i] * m[k];
                else
                    e += kBasis.m[k][i] * m[k];
            }
        d[i] = e + o;
        d[opp(i)] = e - o;
    }
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < MLP_NNC; ++k)
        if (kBasis.m[k][Q - 1] != 0.0f) r += kBasis.m[k][Q - 1] * m[k];
    d[Q - 1] = r;
}

__device__ __forceinline__ short bf16_bits(float f) {
    const __bf16 b = (__bf16)f;
    return __builtin_bit_cast(short, b);
}

// Two and four values at once: one packed conversion per pair (the same rounding as
// bf16_bits, without the repacking of single conversions).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
    const f2v v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ bf4 bf16_quad(acc4 a) {
    const u2v p = {bf16_pair(a[0], a[1]), bf16_pair(a[2], a[3])};
    return __builtin_bit_cast(bf4, p);
}

// relu, then bfloat16: round first, then clamp the bit patterns as int16 (a negative
// bfloat16 is a negative int16, -0 included), one packed max per two values; the same
// result as rounding relu(a) for every finite a
__device__ __forceinline__ bf4 relu_bf16(acc4 a) {
    const bf4 z = {0, 0, 0, 0};
    return __builtin_elementwise_max(bf16_quad(a), z);
}

__device__ __forceinline__ acc4 mfma(bf4 a, bf4 b, acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Two K = 16 steps in one gfx950 K = 32 instruction: A = (a0 | a1), B = (b0 | b1) per lane.
// The contraction pairs the same slot of A and B, so a0 meets b0 and a1 meets b1 whatever the
// instruction's order of k within a lane.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ acc4 mfma2(bf4 a0, bf4 a1, bf4 b0, bf4 b1, acc4 c) {
    typedef short s8v __attribute__((ext_vector_type(8)));
    const s8v a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const s8v b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                   0);
}

// ---------------------------------------------------------------- packing
// Fragment f, lane L, element r (q = L / 16, p = L % 16):
//   forward  0..3   W1 tile o:        A[i=p][k=4q+r] = W1[4q+r][16o+p]
//            4..19  W2 tile (o2, o):  A = W2[16o+4q+r][16o2+p]   (f = 4 + 4 o2 + o)
//            20..23 W3 tile o:        A = W3[16o+4q+r][p]
//   backward 24..27 W3 tile o:        A[i=p][k=4q+r] = W3[16o+p][4q+r]
//            28..43 W2 tile (o1, o2): A = W2[16o1+p][16o2+4q+r]  (f = 28 + 4 o1 + o2)
constexpr int PW1 = 0, PB1 = 1024, PW2 = 1088, PB2 = 5184, PW3 = 5248, PB3 = 6272;
static_assert(PB3 + MLP_NOUT == MLP_PARAMS, "parameter layout");

__device__ __forceinline__ int frag_param(int f, int lane, int r) {
    const int q = lane >> 4, p = lane & 15;
    if (f < 4) return PW1 + (4 * q + r) * 64 + 16 * f + p;
    if (f < 20) {
        const int o2 = (f - 4) >> 2, o = (f - 4) & 3;
        return PW2 + (16 * o + 4 * q + r) * 64 + 16 * o2 + p;
    }
    if (f < 24) return PW3 + (16 * (f - 20) + 4 * q + r) * 16 + p;
    if (f < 28) return PW3 + (16 * (f - 24) + p) * 16 + 4 * q + r;
    const int o1 = (f - 28) >> 2, o2 = (f - 28) & 3;
    return PW2 + (16 * o1 + p) * 64 + 16 * o2 + 4 * q + r;
}

__global__ void __launch_bounds__(64) k_mlp_pack(const float* __restrict__ params, const float* __restrict__ norm,
                                                 float c_guard, MlpPacked* __restrict__ P) {
    const int f = blockIdx.x, lane = threadIdx.x;
    if (f < MLP_NFRAG_ALL) {
#pragma unroll
        for (int r = 0; r < 4; ++r) P->frag[f][lane][r] = (uint16_t)bf16_bits(params[frag_param(f, lane, r)]);
    } else {
        for (int k = lane; k < MLP_NH; k += 64) {
            P->bias[k] = params[PB1 + k];
            P->bias[MLP_NH + k] = params[PB2 + k];
        }
        if (lane < MLP_NOUT) P->bias[2 * MLP_NH + lane] = params[PB3 + lane];
        if (lane < 3 * MLP_NIN) P->norm[lane] = norm[lane];
        if (lane == 0) P->c_guard = c_guard;
        if (lane < 15) P->pad[lane] = 0.0f;
    }
}

// ---------------------------------------------------------------- forward pass
struct FwdW {
    bf4 a1[4], a2[16], a3[4];
    acc4 b1[4], b2[4], b3;
    __device__ __forceinline__ acc4 bias1(int o) const { return b1[o]; }
    __device__ __forceinline__ acc4 bias2(int o) const { return b2[o]; }
    __device__ __forceinline__ acc4 bias3() const { return b3; }
    __device__ __forceinline__ void next_tile() {}
};

__device__ __forceinline__ void load_frags(const MlpPacked* __restrict__ P, bf4 a1[4], bf4 a2[16], bf4 a3[4]) {
    const int lane = threadIdx.x & 63;
    const bf4* fr = (const bf4*)P->frag;
#pragma unroll
    for (int o = 0; o < 4; ++o) a1[o] = fr[(0 + o) * 64 + lane];
#pragma unroll
    for (int o = 0; o < 16; ++o) a2[o] = fr[(4 + o) * 64 + lane];
#pragma unroll
    for (int o = 0; o < 4; ++o) a3[o] = fr[(20 + o) * 64 + lane];
}

__device__ __forceinline__ void load_fwd(const MlpPacked* __restrict__ P, FwdW& W) {
    const int q = (threadIdx.x & 63) >> 4;
    load_frags(P, W.a1, W.a2, W.a3);
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        W.b1[o] = *(const acc4*)(P->bias + 16 * o + 4 * q);
        W.b2[o] = *(const acc4*)(P->bias + MLP_NH + 16 * o + 4 * q);
    }
    W.b3 = *(const acc4*)(P->bias + 2 * MLP_NH + 4 * q);
}

// The same network with the biases read at each use from a workgroup's LDS copy
// (2 * MLP_NH + MLP_NOUT floats; `sb` points at this lane's row group 4q): 36 registers fewer
// per lane.  The pointer is passed through an empty asm statement for every tile, so that the
// compiler reads the biases again instead of keeping them in registers across the tiles.
typedef __attribute__((address_space(3))) const float* lds_cfp;
struct FwdL {
    bf4 a1[4], a2[16], a3[4];
    lds_cfp sb;
    __device__ __forceinline__ acc4 bias1(int o) const { return *(const acc4*)(sb + 16 * o); }
    __device__ __forceinline__ acc4 bias2(int o) const { return *(const acc4*)(sb + MLP_NH + 16 * o); }
    __device__ __forceinline__ acc4 bias3() const { return *(const acc4*)(sb + 2 * MLP_NH); }
    __device__ __forceinline__ void next_tile() { asm volatile("" : "+v"(sb)); }
};

// One 16-cell tile: xb = inputs in B layout (k = feature 4q+r, column = cell p); returns
// the 16 outputs in accumulator layout (row = output 4q+r, column = cell p) and, when
// asked, the two hidden activations in B layout.
template <class W_>
__device__ __forceinline__ acc4 mlp_tile(const W_& W, bf4 xb, bf4 h1[4], bf4 h2[4]) {
#pragma unroll
    for (int o = 0; o < 4; ++o) h1[o] = relu_bf16(mfma(W.a1[o], xb, W.bias1(o)));
#pragma unroll
    for (int o2 = 0; o2 < 4; ++o2) {
        acc4 a = W.bias2(o2);
        a = mfma2(W.a2[4 * o2 + 0], W.a2[4 * o2 + 1], h1[0], h1[1], a);
        a = mfma2(W.a2[4 * o2 + 2], W.a2[4 * o2 + 3], h1[2], h1[3], a);
        h2[o2] = relu_bf16(a);
    }
    acc4 y = W.bias3();
    y = mfma2(W.a3[0], W.a3[1], h2[0], h2[1], y);
    y = mfma2(W.a3[2], W.a3[3], h2[2], h2[3], y);
    return y;
}

// Per-wavefront LDS staging: 64 cells x 16 inputs (bf16) and 64 cells x 16 outputs (fp32).
struct WaveStage {
    short x[64 * 16];
    float y[64 * 16];
};

// Run the network on the 64 cells of this wavefront: in[16] per lane (standardised) ->
// out[16] per lane.  Every lane of the wavefront must call it (matrix cores use all 64).
template <class W_>
__device__ __forceinline__ void mlp_wave(W_& W, WaveStage& S, const float in[16], float out[16]) {
    const int lane = threadIdx.x & 63, q = lane >> 4, p = lane & 15;
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    u4v lo, hi;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo[k] = bf16_pair(in[2 * k], in[2 * k + 1]);
        hi[k] = bf16_pair(in[8 + 2 * k], in[8 + 2 * k + 1]);
    }
    *(u4v*)&S.x[lane * 16] = lo;
    *(u4v*)&S.x[lane * 16 + 8] = hi;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bf4 xb = *(const bf4*)&S.x[(16 * t + p) * 16 + 4 * q];
        W.next_tile();
        bf4 h1[4], h2[4];
        const acc4 y = mlp_tile(W, xb, h1, h2);
        *(acc4*)&S.y[(16 * t + p) * 16 + 4 * q] = y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const acc4 v = *(const acc4*)&S.y[lane * 16 + 4 * k];
        out[4 * k + 0] = v[0];
        out[4 * k + 1] = v[1];
        out[4 * k + 2] = v[2];
        out[4 * k + 3] = v[3];
    }
}

// ---------------------------------------------------------------- closure step
// A channel descriptor read through the constant address space: with a wavefront-uniform
// address the compiler reads it with scalar loads (the descriptors are not written while a
// kernel runs).  Fields that are not used are not loaded.
__device__ __forceinline__ Chan chan_const(const Chan* p) {
    typedef __attribute__((address_space(4))) const uint32_t* cu32_p;
    static_assert(sizeof(Chan) % 4 == 0, "descriptor of whole words");
    Chan c;
    uint32_t* d = (uint32_t*)&c;
    const cu32_p s = (cu32_p)p;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(Chan) / 4); ++k) d[k] = s[k];
    return c;
}

// The lattice step of k_step (pull, moments, Guo-forced BGK, aligned store) with the
// learned correction added before the store.  Workgroups of 256 threads walk the
// segments four at a time with a uniform trip count (the LDS transposes use barriers).
// At most 168 registers: three wavefronts per SIMD.
template <class St, bool NT>
__global__ void __launch_bounds__(256, 3) k_step_cl(LatArgs a, const MlpPacked* __restrict__ P, uint32_t* flags,
                                                 unsigned long long* guarded) {
    using T = typename St::T;
    __shared__ WaveStage stage[4];
    __shared__ float sbias[2 * MLP_NH + MLP_NOUT];
    __shared__ unsigned int blk_bad;
    // the wavefront index as a scalar: segment, channel and its fields then live in scalar
    // registers and are read with scalar loads, which do not wait behind the prefetch
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (threadIdx.x == 0) blk_bad = 0u;  // first read after the barriers of the first pass
    if (threadIdx.x < 2 * MLP_NH + MLP_NOUT) sbias[threadIdx.x] = P->bias[threadIdx.x];  // read after them too
    FwdL W;
    load_frags(P, W.a1, W.a2, W.a3);
    W.sb = (lds_cfp)(sbias + 4 * (lane >> 4));
    // Wait for the weights here: otherwise the first use of each fragment, inside the loop,
    // carries a wait that in later iterations also waits for the prefetch.
#pragma unroll
    for (int o = 0; o < 4; ++o) asm volatile("" ::"v"(W.a1[o]), "v"(W.a3[o]));
#pragma unroll
    for (int o = 0; o < 16; ++o) asm volatile("" ::"v"(W.a2[o]));
    const float* nrm = P->norm;
    const float cg = P->c_guard;
    // The next segment's populations and IB force are loaded one iteration ahead, so that
    // their latency overlaps this segment's network: its populations and the force slot of
    // each cell's tile early in the iteration, the force itself before this segment's stores
    // (a wait for a load issued after the stores would wait for the stores as well).  The
    // segment and channel are wavefront-uniform and read through the constant address space,
    // i.e. with scalar loads, which do not wait behind the vector loads in flight.
    typedef __attribute__((address_space(4))) const int32_t* cint_p;
    // segment of wavefront step sw: its channel and this lane's cell (false past the end)
    auto locate = [&](int64_t sw, int32_t& ci, int32_t& n) -> bool {
        if (sw >= a.nseg) return false;
        const int64_t seg = a.reverse ? a.nseg - 1 - sw : sw;
        ci = ((cint_p)a.seg_ch)[seg];
        const Chan ch = chan_const(a.chan + ci);
        n = (int32_t)((seg - ch.seg_off) * 64 + lane);
        return n < ch.ncell;
    };
    auto load_pops = [&](int32_t ci, int32_t n, int32_t& slot, float r[Q]) {
        const Chan ch = chan_const(a.chan + ci);
        int x, y, z;
        cell_xyz(ch, (uint32_t)n, x, y, z);
        if (a.tile_slot) slot = a.tile_slot[tile_of(ch, x, y, z)];
        pull_loads<St>((const T*)a.src + ch.pop_off, ch, n, x, y, z, r);
    };
    auto load_force = [&](int32_t ci, int32_t n, int32_t slot, float f[3]) {
        if (slot >= 0) {
            const Chan ch = chan_const(a.chan + ci);
            int x, y, z;
            cell_xyz(ch, (uint32_t)n, x, y, z);
            const float* fb = a.force + (int64_t)slot * (3 * TILE_CELLS) + tile_local(x, y, z);
            f[0] = fb[0];
            f[1] = fb[TILE_CELLS];
            f[2] = fb[2 * TILE_CELLS];
        }
    };
    const int64_t stride = (int64_t)gridDim.x * 4;
    int32_t ci_nx = 0, n_nx = 0, slot_nx = -1;
    float r[Q], f_nx[3] = {0.0f, 0.0f, 0.0f};
    bool valid_nx = locate((int64_t)blockIdx.x * 4 + wave, ci_nx, n_nx);
    if (valid_nx) {
        load_pops(ci_nx, n_nx, slot_nx, r);
        load_force(ci_nx, n_nx, slot_nx, f_nx);
    }
    for (int64_t base = (int64_t)blockIdx.x * 4; base < a.nseg; base += stride) {
        const bool valid = valid_nx;
        const int32_t n = n_nx, slot = slot_nx;
        const Chan ch = chan_const(a.chan + ci_nx);
        float g[Q];
        float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
        int x = 0, y = 0, z = 0;
        if (valid) {
            cell_xyz(ch, (uint32_t)n, x, y, z);
#pragma unroll
            for (int i = 0; i < Q; ++i) g[i] = r[i];
            pull_walls(ch, y, g);
            // the channel's force plus the tile's (as ib_force adds them)
            Fx = slot >= 0 ? ch.body[0] + f_nx[0] : ch.body[0];
            Fy = slot >= 0 ? ch.body[1] + f_nx[1] : ch.body[1];
            Fz = slot >= 0 ? ch.body[2] + f_nx[2] : ch.body[2];
        }
        valid_nx = locate(base + stride + wave, ci_nx, n_nx);
        slot_nx = -1;
        if (valid_nx) load_pops(ci_nx, n_nx, slot_nx, r);
        float gn[Q];  // the plain step's post-collision values
        float in[16], mm = 0.0f;
        if (valid) {
            float drho, jx, jy, jz;
            moments(g, drho, jx, jy, jz);
            if (St::onsite && onsite_row(ch, y)) {
                onsite_wall(ch, y, g, Fx, Fy, Fz);
                moments(g, drho, jx, jy, jz);
            }
            const CellState cs = cell_state(drho, jx, jy, jz, Fx, Fy, Fz);
            // g - g^eq feeds both the moments and the collision: one equilibrium per direction
            float d[Q], m[MLP_NNC];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                d[i] = g[i] - geq_c(i, cs);
                gn[i] = bgk_from_neq(i, g[i], d[i], cs, ch.omega, ch.guo);
            }
            to_moments(d, m);
#pragma unroll
            for (int k = 0; k < MLP_NNC; ++k) {
                mm += m[k] * m[k];
                in[k] = (m[k] - nrm[k]) * nrm[16 + k];
            }
            const float ix = Fx - ch.body[0], iy = Fy - ch.body[1], iz = Fz - ch.body[2];
            in[15] = (sqrtf(ix * ix + iy * iy + iz * iz) - nrm[15]) * nrm[31];
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) in[k] = 0.0f;
        }
        float out[16];
        mlp_wave(W, stage[wave], in, out);
        if (valid) {
            float dm[MLP_NNC], dd = 0.0f;
#pragma unroll
            for (int k = 0; k < MLP_NNC; ++k) {
                dm[k] = out[k] * nrm[32 + k];
                dd += dm[k] * dm[k];
            }
            // reject non-finite corrections and |dm| > c |m| (NaN compares false)
            const bool ok = dd <= cg * cg * mm;
            T* dst = (T*)a.dst + ch.pop_off;
            float df[Q];
            from_moments(dm, df);
            if (valid_nx) load_force(ci_nx, n_nx, slot_nx, f_nx);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const float v = ok ? gn[i] + df[i] : gn[i];
                if (NT)
                    St::st_nt(dst + pidx(i, n), v);
                else
                    St::st(dst + pidx(i, n), v);
            }
            const uint64_t bad = __ballot(!ok);
            if (bad && lane == __ffsll((unsigned long long)bad) - 1) atomicAdd(&blk_bad, (unsigned)__popcll(bad));
        } else if (valid_nx) {
            load_force(ci_nx, n_nx, slot_nx, f_nx);
        }
    }
    // one global update per workgroup for the fallback count (the loop is uniform)
    __syncthreads();
    if (threadIdx.x == 0 && blk_bad) {
        atomicOr(flags, LBM_FLAG_CLOSURE_FALLBACK);
        atomicAdd(guarded, (unsigned long long)blk_bad);
    }
}

// ---------------------------------------------------------------- batched forward
// dm[b][k] = y[b][k] * out_scale[k] for standardised raw inputs; B samples, 64 per wave.
__global__ void __launch_bounds__(256) k_mlp_fwd(const MlpPacked* __restrict__ P, const float* __restrict__ raw,
                                                 int64_t B, float* __restrict__ dm) {
    __shared__ WaveStage stage[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    FwdW W;
    load_fwd(P, W);
    const float* nrm = P->norm;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < B; base += (int64_t)gridDim.x * 256) {
        const int64_t b = base + wave * 64 + lane;
        float in[16], out[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) in[k] = b < B ? (raw[b * 16 + k] - nrm[k]) * nrm[16 + k] : 0.0f;
        mlp_wave(W, stage[wave], in, out);
        if (b < B)
#pragma unroll
            for (int k = 0; k < 16; ++k) dm[b * 16 + k] = out[k] * nrm[32 + k];
    }
}

// ---------------------------------------------------------------- training
// One wavefront per workgroup; each takes 64-sample chunks blockIdx, blockIdx + grid, ...
// Loss: sum_b sum_{k<15} (y - t)^2 / (15 B) in standardised units (t = dm / out_scale).
// Output: partial[block][MLP_PARAMS + 1] (gradient, then the loss).
struct TrainLds {
    short xc[64 * 16];    // inputs [cell][in]
    short xT[16 * 64];    // inputs [in][cell]
    float tc[64 * 16];    // standardised targets [cell][out]
    short h1T[64 * 64];   // [hid][cell]
    short h2T[64 * 64];
    short dyT[16 * 64];   // [out][cell]
    short d2T[64 * 64];   // d loss / d a2, [hid][cell]
    short d1T[64 * 64];
    float red[64 * 37];   // bias-gradient / loss reduction
};

__device__ __forceinline__ void put_T(short* T, int row0, int cell, bf4 v) {
    // accumulator / B layout (row row0 + r, column cell) -> [row][cell]
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(row0 + r) * 64 + cell] = v[r];
}

__global__ void __launch_bounds__(64) k_mlp_grad(const MlpPacked* __restrict__ P, const float* __restrict__ raw,
                                                 const float* __restrict__ tgt, int64_t B,
                                                 float* __restrict__ partial) {
    __shared__ TrainLds L;
    const int lane = threadIdx.x, q = lane >> 4, p = lane & 15;
    FwdW W;
    load_fwd(P, W);
    const bf4* fr = (const bf4*)P->frag;
    const float* nrm = P->norm;
    const float gscale = 2.0f / (15.0f * (float)B);
    acc4 gW1[4], gW2[16], gW3[4];
    acc4 gb1[4], gb2[4], gb3;
    const acc4 z4 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int o = 0; o < 4; ++o) gW1[o] = gW3[o] = gb1[o] = gb2[o] = z4;
#pragma unroll
    for (int o = 0; o < 16; ++o) gW2[o] = z4;
    gb3 = z4;
    float lsum = 0.0f;
    const int64_t nchunk = (B + 63) / 64;
    for (int64_t chunk = blockIdx.x; chunk < nchunk; chunk += gridDim.x) {
        const int64_t b = chunk * 64 + lane;
        const bool v = b < B;
        // stage inputs (both layouts) and targets
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float xv = v ? (raw[b * 16 + k] - nrm[k]) * nrm[16 + k] : 0.0f;
            const short xs = bf16_bits(xv);
            L.xc[lane * 16 + k] = xs;
            L.xT[k * 64 + lane] = xs;
            L.tc[lane * 16 + k] = (v && k < MLP_NNC) ? tgt[b * 16 + k] / nrm[32 + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < 4; ++t) {
            const int cell = 16 * t + p;
            const bool cv = chunk * 64 + cell < B;
            const bf4 xb = *(const bf4*)&L.xc[cell * 16 + 4 * q];
            bf4 h1[4], h2[4];
            const acc4 y = mlp_tile(W, xb, h1, h2);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                put_T(L.h1T, 16 * o + 4 * q, cell, h1[o]);
                put_T(L.h2T, 16 * o + 4 * q, cell, h2[o]);
            }
            // d loss / d y (row = output 4q + r, column = cell)
            const acc4 tt = *(const acc4*)&L.tc[cell * 16 + 4 * q];
            acc4 dy;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float e = (cv && 4 * q + r < MLP_NNC) ? y[r] - tt[r] : 0.0f;
                lsum += e * e;
                dy[r] = gscale * e;
            }
            gb3 += dy;
            const bf4 dyb = bf16_quad(dy);
            put_T(L.dyT, 4 * q, cell, dyb);
            // d / d a2 = (W3 dy) * [a2 > 0]
            bf4 d2[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                acc4 a = mfma(fr[(24 + o) * 64 + lane], dyb, z4);
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = h2[o][r] > 0 ? a[r] : 0.0f;  // bf16 > 0 as int16 > 0
                gb2[o] += a;
                d2[o] = bf16_quad(a);
                put_T(L.d2T, 16 * o + 4 * q, cell, d2[o]);
            }
            // d / d a1 = (W2 d2) * [a1 > 0]
#pragma unroll
            for (int o1 = 0; o1 < 4; ++o1) {
                acc4 a = z4;
#pragma unroll
                for (int o2 = 0; o2 < 4; ++o2) a = mfma(fr[(28 + 4 * o1 + o2) * 64 + lane], d2[o2], a);
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = h1[o1][r] > 0 ? a[r] : 0.0f;
                gb1[o1] += a;
                const bf4 d1 = bf16_quad(a);
                put_T(L.d1T, 16 * o1 + 4 * q, cell, d1);
            }
        }
        __syncthreads();
        // weight gradients: contractions over the 64 cells of the chunk (4 k-steps)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            const int c0 = 16 * kc + 4 * q;
            const bf4 xa = *(const bf4*)&L.xT[p * 64 + c0];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const bf4 d1b = *(const bf4*)&L.d1T[(16 * o + p) * 64 + c0];
                gW1[o] = mfma(xa, d1b, gW1[o]);  // dW1[in][hid1]
            }
            const bf4 dyb = *(const bf4*)&L.dyT[p * 64 + c0];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const bf4 h2a = *(const bf4*)&L.h2T[(16 * o + p) * 64 + c0];
                gW3[o] = mfma(h2a, dyb, gW3[o]);  // dW3[hid2][out]
            }
#pragma unroll
            for (int o1 = 0; o1 < 4; ++o1) {
                const bf4 h1a = *(const bf4*)&L.h1T[(16 * o1 + p) * 64 + c0];
#pragma unroll
                for (int o2 = 0; o2 < 4; ++o2) {
                    const bf4 d2b = *(const bf4*)&L.d2T[(16 * o2 + p) * 64 + c0];
                    gW2[4 * o1 + o2] = mfma(h1a, d2b, gW2[4 * o1 + o2]);  // dW2[hid1][hid2]
                }
            }
        }
        __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * (MLP_PARAMS + 1);
    // weight gradients: accumulator row 4q + r, column p
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            out[PW1 + (4 * q + r) * 64 + 16 * o + p] = gW1[o][r];
            out[PW3 + (16 * o + 4 * q + r) * 16 + p] = gW3[o][r];
        }
#pragma unroll
        for (int o1 = 0; o1 < 4; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 4; ++o2)
                out[PW2 + (16 * o1 + 4 * q + r) * 64 + 16 * o2 + p] = gW2[4 * o1 + o2][r];
    }
    // bias gradients and loss: sum over the 16 lanes (cells) of each row group, fixed order
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            L.red[lane * 37 + 4 * o + r] = gb1[o][r];
            L.red[lane * 37 + 16 + 4 * o + r] = gb2[o][r];
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) L.red[lane * 37 + 32 + r] = gb3[r];
    L.red[lane * 37 + 36] = lsum;
    __syncthreads();
    {
        // lane -> hidden unit h = lane: row group q' = (h % 16) / 4, element (o, r) = (h / 16, h % 4)
        const int h = lane, o = h >> 4, qq = (h & 15) >> 2, r = h & 3;
        float s1 = 0.0f, s2 = 0.0f;
        for (int c = 0; c < 16; ++c) {
            s1 += L.red[(16 * qq + c) * 37 + 4 * o + r];
            s2 += L.red[(16 * qq + c) * 37 + 16 + 4 * o + r];
        }
        out[PB1 + h] = s1;
        out[PB2 + h] = s2;
        if (h < MLP_NOUT) {
            float s3 = 0.0f;
            for (int c = 0; c < 16; ++c) s3 += L.red[(16 * (h >> 2) + c) * 37 + 32 + (h & 3)];
            out[PB3 + h] = s3;
        }
        if (h == 0) {
            float s = 0.0f;
            for (int c = 0; c < 64; ++c) s += L.red[c * 37 + 36];
            out[MLP_PARAMS] = s / (15.0f * (float)B);
        }
    }
}

// Sum the per-workgroup partials in a fixed order (double accumulation): slice k of
// RD_SLICES holds consecutive workgroups, summed in workgroup order by one thread, and the
// slices are then added in slice order, so the result does not depend on scheduling.  A
// workgroup covers RD_P parameters (coalesced rows) with all slices in parallel.
constexpr int RD_P = 64, RD_SLICES = 16;
__global__ void __launch_bounds__(RD_P * RD_SLICES) k_grad_reduce(const float* __restrict__ partial, int nblk,
                                                               float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ double part[RD_SLICES][RD_P];
    const int p = threadIdx.x % RD_P, sl = threadIdx.x / RD_P;
    const int j = blockIdx.x * RD_P + p;
    const int per = (nblk + RD_SLICES - 1) / RD_SLICES;
    const int b0 = sl * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    double s = 0.0;
    if (j <= MLP_PARAMS) {
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            float t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = partial[(int64_t)(b + u) * (MLP_PARAMS + 1) + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += t[u];
        }
        for (; b < b1; ++b) s += partial[(int64_t)b * (MLP_PARAMS + 1) + j];
    }
    part[sl][p] = s;
    __syncthreads();
    if (sl == 0 && j <= MLP_PARAMS) {
        double tot = 0.0;
        for (int k = 0; k < RD_SLICES; ++k) tot += part[k][p];
        if (j < MLP_PARAMS)
            grad[j] = (float)tot;
        else if (loss)
            *loss = (float)tot;
    }
}

// Adam (Kingma & Ba 2015) with bias correction; step counts from 1.
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    th[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// Input mean / scale and output scale over B samples: partial sums per workgroup in
// double, then a fixed-order final pass.  in_scale = 1/std (1 where std = 0), out_scale =
// root mean square of the target (1 where 0).
__global__ void __launch_bounds__(256) k_norm_partial(const float* __restrict__ raw, const float* __restrict__ tgt,
                                                      int64_t B, double* __restrict__ part) {
    __shared__ double red[256];
    const int col = threadIdx.x & 15, sub = threadIdx.x >> 4;  // 16 rows per pass
    double s = 0.0, s2 = 0.0, t2 = 0.0;
    for (int64_t b = (int64_t)blockIdx.x * 16 + sub; b < B; b += (int64_t)gridDim.x * 16) {
        const double x = raw[b * 16 + col], t = tgt[b * 16 + col];
        s += x;
        s2 += x * x;
        t2 += t * t;
    }
    double* out = part + (int64_t)blockIdx.x * 48;
    const double vals[3] = {s, s2, t2};
    for (int k = 0; k < 3; ++k) {
        red[threadIdx.x] = vals[k];
        __syncthreads();
        if (sub == 0) {
            double a = 0.0;
            for (int r = 0; r < 16; ++r) a += red[r * 16 + col];
            out[16 * k + col] = a;
        }
        __syncthreads();
    }
}

__global__ void k_norm_final(const double* __restrict__ part, int nblk, int64_t B, float* __restrict__ norm) {
    const int col = threadIdx.x;
    if (col >= 16) return;
    double s = 0.0, s2 = 0.0, t2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s += part[b * 48 + col];
        s2 += part[b * 48 + 16 + col];
        t2 += part[b * 48 + 32 + col];
    }
    const double mean = s / (double)B;
    const double var = s2 / (double)B - mean * mean;
    const double sd = var > 0.0 ? sqrt(var) : 0.0;
    const double rms = sqrt(t2 / (double)B);
    norm[col] = (float)mean;
    norm[16 + col] = sd > 0.0 ? (float)(1.0 / sd) : 1.0f;
    norm[32 + col] = rms > 0.0 ? (float)rms : 1.0f;
}

// ---------------------------------------------------------------- training data
// 2x restriction of a fine channel (acoustic scaling dt_c = 2 dt_f) into coarse shifted
// pre-collision populations (paper order [19][Nc]) and the coarse IB force density
// ([3][Nc], twice the block mean of the fine IB force):
//   rho_c, j_c = block means;  g_c = geq(rho_c, j_c / rho_c) + (2 tau_c / tau_f) mean(g - geq(rho, j / rho)).
template <class St>
__global__ void __launch_bounds__(256) k_restrict(LatArgs a, float resc, float* __restrict__ gc,
                                                  float* __restrict__ Fc) {
    using T = typename St::T;
    const Chan& ch = a.chan[0];
    const int NX = ch.nx >> 1, NY = ch.ny >> 1, NZ = ch.nz >> 1;
    const int64_t Nc = (int64_t)NX * NY * NZ;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Nc) return;
    const int X = (int)(c % NX), Y = (int)((c / NX) % NY), Z = (int)(c / ((int64_t)NX * NY));
    const T* s = (const T*)a.src + ch.pop_off;
    float sum_dr = 0.0f, sjx = 0.0f, sjy = 0.0f, sjz = 0.0f, sfx = 0.0f, sfy = 0.0f, sfz = 0.0f;
    float neq[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) neq[i] = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const int x = 2 * X + (k & 1), y = 2 * Y + ((k >> 1) & 1), z = 2 * Z + (k >> 2);
        const int32_t n = x + ch.nx * (y + ch.ny * z);
        float g[Q];
        pull<St>(s, ch, ch.ncell, n, x, y, z, g);
        float dr, jx, jy, jz, Fx, Fy, Fz;
        moments(g, dr, jx, jy, jz);
        const float ir = 1.0f / (1.0f + dr);
#pragma unroll
        for (int i = 0; i < Q; ++i) neq[i] += g[i] - geq_i(i, dr, jx * ir, jy * ir, jz * ir);
        sum_dr += dr;
        sjx += jx;
        sjy += jy;
        sjz += jz;
        ib_force(a, ch, x, y, z, Fx, Fy, Fz);
        sfx += Fx - ch.body[0];
        sfy += Fy - ch.body[1];
        sfz += Fz - ch.body[2];
    }
    const float dr = 0.125f * sum_dr, ir = 1.0f / (1.0f + dr);
    const float ux = 0.125f * sjx * ir, uy = 0.125f * sjy * ir, uz = 0.125f * sjz * ir;
#pragma unroll
    for (int i = 0; i < Q; ++i) gc[(int64_t)i * Nc + c] = geq_i(i, dr, ux, uy, uz) + resc * 0.125f * neq[i];
    Fc[c] = 0.25f * sfx;
    Fc[Nc + c] = 0.25f * sfy;
    Fc[2 * Nc + c] = 0.25f * sfz;
}

// Features and targets of one coarse step: collide g0 (Guo-forced BGK with force
// body + F_IB), invert the streaming of g1, project the difference on M_nc.
// feat[n] = (m_neq[15], |F_IB|), target[n] = (dm[15], 0).
__global__ void __launch_bounds__(256) k_targets(Chan ch, const float* __restrict__ g0, const float* __restrict__ F,
                                                 const float* __restrict__ g1, float* __restrict__ feat,
                                                 float* __restrict__ target) {
    const int64_t N = ch.ncell;
    const int64_t nn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nn >= N) return;
    const int32_t n = (int32_t)nn;
    int x, y, z;
    cell_xyz(ch, (uint32_t)n, x, y, z);
    float g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = g0[(int64_t)i * N + n];
    float drho, jx, jy, jz;
    moments(g, drho, jx, jy, jz);
    const float fx = F[n], fy = F[N + n], fz = F[2 * N + n];
    const CellState cs = cell_state(drho, jx, jy, jz, ch.body[0] + fx, ch.body[1] + fy, ch.body[2] + fz);
    float d[Q], e[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float bgk = bgk_c(i, g[i], cs, ch.omega, ch.guo);
        int32_t m;
        const float tgt = step_out(ch, i, x, y, z, m) ? g1[(int64_t)i * N + m]
                                                      : g1[(int64_t)opp(i) * N + n] + wall_term(ch, i);
        d[i] = g[i] - geq_c(i, cs);
        e[i] = tgt - bgk;
    }
    float mf[MLP_NNC], mt[MLP_NNC];
    to_moments(d, mf);
    to_moments(e, mt);
#pragma unroll
    for (int k = 0; k < MLP_NNC; ++k) {
        feat[nn * 16 + k] = mf[k];
        target[nn * 16 + k] = mt[k];
    }
    feat[nn * 16 + 15] = sqrtf(fx * fx + fy * fy + fz * fz);
    target[nn * 16 + 15] = 0.0f;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_mlp_pack(hipStream_t s, const float* params, const float* norm, float c_guard, MlpPacked* P) {
    k_mlp_pack<<<dim3(MLP_NFRAG_ALL + 1), dim3(64), 0, s>>>(params, norm, c_guard, P);
    return hipGetLastError();
}

template <class St>
static hipError_t step_cl_typed(lbm_ctx* c, const LatArgs& a) {
    // 8 workgroups per CU (three of them resident at a time); where that would leave each
    // workgroup fewer than two passes over its four segments, 3 per CU, so that the loads of a
    // next segment issued during each pass find one
    const int64_t units = (c->total_segs + 3) / 4;
    const int64_t wide = c->ib_grid * 2, resident = c->ib_grid * 3 / 4;
    int64_t grid = units >= 2 * wide ? wide : resident;
    if (grid > units) grid = units;
    unsigned long long* cnt = (unsigned long long*)(c->d_flags + 2);
    if (c->launch.nontemporal)
        k_step_cl<St, true><<<dim3((unsigned)grid), dim3(256), 0, c->stream>>>(a, c->d_mlp, c->d_flags, cnt);
    else
        k_step_cl<St, false><<<dim3((unsigned)grid), dim3(256), 0, c->stream>>>(a, c->d_mlp, c->d_flags, cnt);
    return hipGetLastError();
}

hipError_t launch_step_closure(lbm_ctx* c, const LatArgs& a) {
    return with_storage(c, [&](auto st) { return step_cl_typed<decltype(st)>(c, a); });
}

hipError_t launch_mlp_forward(hipStream_t s, const MlpPacked* P, const float* raw, int64_t B, float* dm,
                              int64_t grid_max) {
    int64_t grid = (B + 255) / 256;
    if (grid > grid_max) grid = grid_max;
    if (grid < 1) return hipSuccess;
    k_mlp_fwd<<<dim3((unsigned)grid), dim3(256), 0, s>>>(P, raw, B, dm);
    return hipGetLastError();
}

int64_t mlp_grad_blocks(int64_t B, int64_t grid_max) {
    int64_t nb = (B + 63) / 64;
    return nb < grid_max ? nb : grid_max;
}

hipError_t launch_mlp_grad(hipStream_t s, const MlpPacked* P, const float* raw, const float* tgt, int64_t B,
                           float* partial, int64_t nblk, float* grad, float* loss) {
    k_mlp_grad<<<dim3((unsigned)nblk), dim3(64), 0, s>>>(P, raw, tgt, B, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_grad_reduce<<<dim3((MLP_PARAMS + 1 + RD_P - 1) / RD_P), dim3(RD_P * RD_SLICES), 0, s>>>(partial, (int)nblk, grad,
                                                                                          loss);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, float* th, const float* g, float* m, float* v, int64_t n, int step, float lr,
                       float b1, float b2, float eps) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    k_adam<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(th, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_norm(hipStream_t s, const float* raw, const float* tgt, int64_t B, double* part, int nblk,
                       float* norm) {
    k_norm_partial<<<dim3(nblk), dim3(256), 0, s>>>(raw, tgt, B, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_norm_final<<<dim3(1), dim3(64), 0, s>>>(part, nblk, B, norm);
    return hipGetLastError();
}

hipError_t launch_restrict(lbm_ctx* c, const LatArgs& a, float resc, float* gc, float* Fc) {
    const Chan& ch = c->chans[0];
    const int64_t Nc = (int64_t)(ch.nx / 2) * (ch.ny / 2) * (ch.nz / 2);
    const dim3 g((unsigned)((Nc + 255) / 256)), b(256);
    switch (c->storage) {
        case LBM_STORE_F32: k_restrict<StF32><<<g, b, 0, c->stream>>>(a, resc, gc, Fc); break;
        case LBM_STORE_F16: k_restrict<StF16><<<g, b, 0, c->stream>>>(a, resc, gc, Fc); break;
        case LBM_STORE_BF16: k_restrict<StBF16><<<g, b, 0, c->stream>>>(a, resc, gc, Fc); break;
    }
    return hipGetLastError();
}

hipError_t launch_targets(hipStream_t s, const Chan& ch, const float* g0, const float* F, const float* g1,
                          float* feat, float* target) {
    k_targets<<<dim3((unsigned)((ch.ncell + 255) / 256)), dim3(256), 0, s>>>(ch, g0, F, g1, feat, target);
    return hipGetLastError();
}

}  // namespace lbmib
