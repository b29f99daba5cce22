// adhesion.hip -- stochastic adhesion of platelet receptors to wall ligands (section 3.2,
// Eq. (12)-(14)): the ligand table by wall cell, and the Monte-Carlo step (breaks, bids,
// acceptance).  The bond forces are gathered per node with the other membrane forces (ib.hip).
//
// One step at the positions after the move:
//   k_adh_receptors  one thread per receptor point: its position from its triangle; two
//                    uniforms from Philox4x32-10 (counter = receptor, step); a bond present at
//                    the start breaks with P_r (Bell off-rate, Eq. (12)); a receptor unbound at
//                    the start looks up the ligands in the 3 x 3 wall cells around it, takes the
//                    nearest one in reach that had fewer than four bonds at the start (lower id on
//                    a tie) and bids for it with P_f (Eq. (13));
//   k_adh_ligands    one thread per ligand: bonds after this step's breaks, then its bids in
//                    ascending receptor id up to four bonds; clears the step's scratch and
//                    advances the step counter.
// The start-of-step counts are not written during the first kernel (breaks and bids go to
// scratch), so every receptor sees the same state whatever the scheduling.  A bid list holds
// ADH_MAX_BIDS bids; more in one step are dropped and counted (the flag LBM_FLAG_ADHESION_BIDS).
#include "lbm_internal.h"

namespace lbmib {

namespace {

// Scratch layout (int32 words) of ib_membrane::adh_work.
struct AdhWork {
    unsigned long long* step;  // [1] Monte-Carlo steps done
    int32_t* lost;             // [1] bids dropped from a full list
    int32_t* broken;           // [nl] bonds broken this step
    int32_t* nbid;             // [nl] bids received this step
    int32_t* cell_lig;         // [nl] ligand ids ordered by wall cell
    int32_t* bids;             // [nl][ADH_MAX_BIDS]
    int32_t* cell_ptr;         // [cells + 1]
    int32_t* cell_fill;        // [cells + 1]
};

__host__ __device__ inline int adh_cells(double extent, double capture) {
    const double c = floor(extent / capture);
    return c < 1.0 ? 1 : (int)c;
}

__host__ __device__ inline AdhWork adh_work(const ib_membrane& m) {
    const int64_t nl = m.adh_nl;
    const int64_t cells = (int64_t)adh_cells(m.adh_nx, m.adh_capture) * adh_cells(m.adh_nz, m.adh_capture);
    int32_t* w = m.adh_work;
    AdhWork a;
    a.step = (unsigned long long*)w;
    a.lost = w + 2;
    a.broken = w + 8;
    a.nbid = w + 8 + nl;
    a.cell_lig = w + 8 + 2 * nl;
    a.bids = w + 8 + 3 * nl;
    a.cell_ptr = w + 8 + nl * (3 + ADH_MAX_BIDS);
    a.cell_fill = a.cell_ptr + cells + 1;
    return a;
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011): ten rounds of two 32x32 -> 64-bit
// multiplications with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// A double in [0, 1): the top 27 bits of `a` above the top 26 bits of `b`.
__device__ __forceinline__ double unit53(uint32_t a, uint32_t b) {
    return (double)(a >> 5) * 0x1p-27 + (double)(b >> 6) * 0x1p-53;
}

// Cell of a wall point (x, z) (wrapped into the periodic box).
__device__ __forceinline__ void wall_cell(const ib_membrane& m, double x, double z, int gx, int gz, int& cx,
                                          int& cz) {
    double xw = fmod(x, m.adh_nx);
    if (xw < 0.0) xw += m.adh_nx;
    double zw = fmod(z, m.adh_nz);
    if (zw < 0.0) zw += m.adh_nz;
    cx = (int)floor(xw / m.adh_nx * gx);
    cz = (int)floor(zw / m.adh_nz * gz);
    cx = cx < 0 ? 0 : (cx >= gx ? gx - 1 : cx);
    cz = cz < 0 ? 0 : (cz >= gz ? gz - 1 : cz);
}

// Receptor minus ligand, x and z by the minimum image.  Products and sums are rounded one at a
// time (no fused multiply-adds), as the reference evaluates them.
__device__ __forceinline__ double adh_sep(const ib_membrane& m, const double xr[3], int64_t l, double d[3]) {
    double dx = xr[0] - m.lig_xz[2 * l];
    double dz = xr[2] - m.lig_xz[2 * l + 1];
    dx = __dsub_rn(dx, __dmul_rn(m.adh_nx, rint(dx / m.adh_nx)));
    dz = __dsub_rn(dz, __dmul_rn(m.adh_nz, rint(dz / m.adh_nz)));
    d[0] = dx;
    d[1] = xr[1] - m.adh_wall_y;
    d[2] = dz;
    return sqrt(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(d[1], d[1])), __dmul_rn(dz, dz)));
}

__device__ __forceinline__ void receptor_pos(const ib_membrane& m, const double* X, int64_t r, double xr[3]) {
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s = __dadd_rn(s, __dmul_rn(m.rec_bary[3 * r + k], X[c * m.n + m.rec_tri[3 * r + k]]));
        xr[c] = s;
    }
}

// ---------------------------------------------------------------- ligand table (set-up)
__global__ void k_adh_cell_count(ib_membrane m, int gx, int gz) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= m.adh_nl) return;
    int cx, cz;
    wall_cell(m, m.lig_xz[2 * l], m.lig_xz[2 * l + 1], gx, gz, cx, cz);
    atomicAdd(&adh_work(m).cell_fill[(int64_t)cz * gx + cx], 1);
}

// Exclusive scan of the cell counts (one workgroup), then the fill counters back to zero.
__global__ void __launch_bounds__(1024) k_adh_cell_scan(ib_membrane m, int64_t cells) {
    __shared__ int32_t part[1024];
    const AdhWork w = adh_work(m);
    const int64_t per = (cells + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = lo + per < cells ? lo + per : cells;
    int32_t s = 0;
    for (int64_t c = lo; c < hi; ++c) s += w.cell_fill[c];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int32_t v = part[t];
            part[t] = run;
            run += v;
        }
        w.cell_ptr[cells] = run;
    }
    __syncthreads();
    int32_t run = part[threadIdx.x];
    for (int64_t c = lo; c < hi; ++c) {
        const int32_t v = w.cell_fill[c];
        w.cell_ptr[c] = run;
        run += v;
        w.cell_fill[c] = 0;
    }
}

// Ligands into their cells (the order inside a cell does not matter: the lookup takes the
// nearest ligand and the lower id on a tie).
__global__ void k_adh_cell_fill(ib_membrane m, int gx, int gz) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= m.adh_nl) return;
    const AdhWork w = adh_work(m);
    int cx, cz;
    wall_cell(m, m.lig_xz[2 * l], m.lig_xz[2 * l + 1], gx, gz, cx, cz);
    const int64_t c = (int64_t)cz * gx + cx;
    w.cell_lig[w.cell_ptr[c] + atomicAdd(&w.cell_fill[c], 1)] = (int32_t)l;
}

// ---------------------------------------------------------------- Monte-Carlo step
__global__ void __launch_bounds__(256) k_adh_receptors(ib_membrane m, const double* X, int gx, int gz) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m.adh_nr) return;
    const AdhWork w = adh_work(m);
    const unsigned long long step = *w.step;
    // the step's four words for this receptor (drawn only where a test is made)
    uint32_t c[4] = {(uint32_t)r, (uint32_t)step, (uint32_t)(step >> 32), 0u};
    double xr[3], d[3];
    receptor_pos(m, X, r, xr);
    const int32_t b = m.bond[r];
    if (b >= 0) {
        philox4x32_10(c, (uint32_t)m.adh_seed, (uint32_t)(m.adh_seed >> 32));
        const double L = adh_sep(m, xr, b, d);
        const double Fb = m.adh_sigma * fabs(L - m.adh_lb);
        const double koff = m.adh_koff0 * exp(m.adh_gamma * Fb / m.adh_kT);
        if (unit53(c[0], c[1]) < 1.0 - exp(-koff)) {
            m.bond[r] = -1;
            atomicAdd(&w.broken[b], 1);
        }
        return;
    }
    if (!(fabs(xr[1] - m.adh_wall_y) < m.adh_capture)) return;
    int cx, cz;
    wall_cell(m, xr[0], xr[2], gx, gz, cx, cz);
    int64_t best = -1;
    double bd = 0.0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int ox = -1; ox <= 1; ++ox) {
            const int ccx = (cx + ox + gx) % gx, ccz = (cz + oz + gz) % gz;
            const int64_t cell = (int64_t)ccz * gx + ccx;
            for (int32_t p = w.cell_ptr[cell]; p < w.cell_ptr[cell + 1]; ++p) {
                const int64_t l = w.cell_lig[p];
                if (m.lig_count[l] >= 4) continue;
                const double L = adh_sep(m, xr, l, d);
                if (!(L < m.adh_capture)) continue;
                if (best < 0 || L < bd || (L == bd && l < best)) {
                    best = l;
                    bd = L;
                }
            }
        }
    if (best < 0) return;
    philox4x32_10(c, (uint32_t)m.adh_seed, (uint32_t)(m.adh_seed >> 32));
    const double s = fabs(bd - m.adh_lb);
    const double kon = m.adh_kon0 * exp(m.adh_sigma * s * (m.adh_gamma - 0.5 * s) / m.adh_kT);
    if (unit53(c[2], c[3]) < 1.0 - exp(-kon)) {
        const int slot = atomicAdd(&w.nbid[best], 1);
        if (slot < ADH_MAX_BIDS)
            w.bids[best * ADH_MAX_BIDS + slot] = (int32_t)r;
        else
            atomicAdd(w.lost, 1);
    }
}

__global__ void __launch_bounds__(256) k_adh_ligands(ib_membrane m, uint32_t* flags) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const AdhWork w = adh_work(m);
    if (l == 0) {
        *w.step += 1ull;
        if (flags && *w.lost > 0) atomicOr(flags, LBM_FLAG_ADHESION_BIDS);
    }
    if (l >= m.adh_nl) return;
    int32_t cnt = m.lig_count[l] - w.broken[l];
    int nb = w.nbid[l];
    nb = nb < ADH_MAX_BIDS ? nb : ADH_MAX_BIDS;
    int32_t* bl = w.bids + l * ADH_MAX_BIDS;
    // accept the lowest receptor ids first: repeated minimum over the (short) list
    for (int taken = 0; taken < nb && cnt < 4; ++taken) {
        int at = taken;
        for (int j = taken + 1; j < nb; ++j)
            if (bl[j] < bl[at]) at = j;
        const int32_t r = bl[at];
        bl[at] = bl[taken];
        bl[taken] = r;
        m.bond[r] = (int32_t)l;
        ++cnt;
    }
    m.lig_count[l] = cnt;
    w.broken[l] = 0;
    w.nbid[l] = 0;
}

}  // namespace

bool adhesion_on(const ib_membrane& m) { return m.adh_nr > 0 && m.adh_nl > 0; }

int64_t adhesion_work_ints(int64_t nl, double nx, double nz, double capture) {
    const int64_t cells = (int64_t)adh_cells(nx, capture) * adh_cells(nz, capture);
    return 8 + nl * (3 + ADH_MAX_BIDS) + 2 * (cells + 1);
}

hipError_t launch_adhesion_setup(const ib_membrane* m, hipStream_t s) {
    if (!adhesion_on(*m)) return hipSuccess;
    const int gx = adh_cells(m->adh_nx, m->adh_capture), gz = adh_cells(m->adh_nz, m->adh_capture);
    const int64_t cells = (int64_t)gx * gz;
    const int64_t words = adhesion_work_ints(m->adh_nl, m->adh_nx, m->adh_nz, m->adh_capture);
    hipError_t e = launch_fill_i32(s, m->adh_work, words, 0);
    if (e != hipSuccess) return e;
    const dim3 g((unsigned)((m->adh_nl + 255) / 256)), b(256);
    k_adh_cell_count<<<g, b, 0, s>>>(*m, gx, gz);
    k_adh_cell_scan<<<dim3(1), dim3(1024), 0, s>>>(*m, cells);
    k_adh_cell_fill<<<g, b, 0, s>>>(*m, gx, gz);
    return hipGetLastError();
}

hipError_t launch_adhesion_step(const ib_membrane* m, const double* X, uint32_t* flags, hipStream_t s) {
    if (!adhesion_on(*m)) return hipSuccess;
    const int gx = adh_cells(m->adh_nx, m->adh_capture), gz = adh_cells(m->adh_nz, m->adh_capture);
    k_adh_receptors<<<dim3((unsigned)((m->adh_nr + 255) / 256)), dim3(256), 0, s>>>(*m, X, gx, gz);
    k_adh_ligands<<<dim3((unsigned)((m->adh_nl + 255) / 256)), dim3(256), 0, s>>>(*m, flags);
    return hipGetLastError();
}

}  // namespace lbmib
