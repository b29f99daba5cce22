/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice-Boltzmann + immersed-boundary library.
 *
 * The library implements the data-parallel core of the platelet / blood-flow model of
 * Wu, Xu, Kim & Alber (arXiv:1312.2234): a D3Q19 BGK lattice-Boltzmann step with the
 * Guo body-force term (section 3.3, Eq. (16)-(21)), coupled to Lagrangian membrane
 * nodes by the immersed-boundary method (section 3.4.2, Eq. (33)-(36)), in the
 * per-step order of Fig. 1: membrane forces -> spread -> LBM -> interpolate -> move.
 *
 * Conventions shared by every call
 *   Units        lattice units: h = dt = rho_0 = 1.
 *   Geometry     x and z periodic; y bounded by two walls (halfway bounce-back) at the
 *                planes y = -1/2 and y = ny - 1/2 when `walls` = 1; by the on-site
 *                velocity walls of Eq. (23)-(30) on the rows y = 0 and y = ny - 1 when
 *                `walls` = 2; periodic when 0.
 *   Numbering    D3Q19 directions in the paper's order i = 1..19 (stored 0..18), the
 *                order fixed by the on-site wall equations Eq. (23)-(30).
 *   Layout       SoA, x fastest: cell n = x + nx*(y + ny*z).  Per-cell fields of all
 *                channels are concatenated in channel order (channel c starts at the sum
 *                of the cell counts of channels < c); vector fields are [3][cells] per
 *                channel.  Lagrangian arrays are SoA [3][n] (X in float64, F/U float32);
 *                nodes of all channels concatenated in channel order.
 *   Memory       every pointer argument except where marked "host" is DEVICE memory owned
 *                by the caller.  The library never allocates device memory: the caller
 *                provides one workspace of lbm_workspace_bytes() bytes to lbm_create() and
 *                keeps it alive until lbm_destroy().  The library owns only the small host
 *                handle, and one fixed device array per GPU that mlp_grad_noalloc uses.
 *   Streams      every call only enqueues work on the context's stream (a hipStream_t
 *                passed as void*); outputs are valid after that stream synchronises.
 *                Calls that return data to the host (lbm_error_flags) synchronise it.
 *   Errors       host-side validation returns LBM_ERR_ARG (null pointer, bad size, tau <=
 *                1/2, wall-normal wall velocity, workspace too small, node count above the
 *                capacity given at create time); a failed HIP launch returns LBM_ERR_HIP;
 *                calls in the wrong order return LBM_ERR_STATE.  Nothing is thrown across
 *                the ABI.  Conditions only the device can see (an IB node outside the
 *                wall band, a non-finite force) set bits read by lbm_error_flags(); the
 *                kernels clamp indices so that they never access memory out of bounds.
 *   Threads      a context is used by one host thread at a time.
 */
#ifndef MI355_LBMIB_H
#define MI355_LBMIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque host handle */

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = 1,
    LBM_ERR_STATE = 2,
    LBM_ERR_HIP = 3,
    LBM_ERR_UNSUPPORTED = 4
} lbm_status;

/* Storage of the populations.  All forms store the weight-shifted value g_i = f_i - w_i
 * and compute in float32; F16 / BF16 halve the bytes per update (round to nearest even
 * on store). */
typedef enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2 } lbm_storage;

/* Discrete delta kernel phi of Eq. (35): the cosine kernel of Eq. (36) (zero for
 * |r| >= 2), or Peskin's 4-point kernel. */
typedef enum { IB_PHI_COS4 = 0, IB_PHI_PESKIN4 = 1 } ib_kernel;

/* Error bits reported by lbm_error_flags(). */
#define LBM_FLAG_NODE_OUTSIDE 0x1u  /* an IB node's y fell outside [-1, ny) ([0, ny-1] with on-site
                                       walls), or was not finite */
#define LBM_FLAG_LIST_OVERFLOW 0x2u /* IB tile lists exceeded their capacity (contributions lost) */
#define LBM_FLAG_FORCE_NONFINITE 0x4u /* a Lagrangian force was Inf/NaN (force field set to NaN) */
#define LBM_FLAG_CLOSURE_FALLBACK 0x8u /* the learned closure fell back to plain BGK at some node */
#define LBM_FLAG_REBIN_MARGIN 0x20u /* with lbm_launch.rebin > 1, a node left the margin it was
                                        binned with before the next binning */
#define LBM_FLAG_ADHESION_BIDS 0x10u /* a ligand received more adhesion bids in one step than its bid
                                        list holds (ADH_MAX_BIDS): some were dropped */

/* One channel (an independent lattice).  Section 3.3: lattice size, relaxation time tau
 * (Eq. (16), viscosity (tau - 1/2)/3 by Eq. (22)), constant body force added to the IB
 * force in Eq. (19), wall velocities of the two y-walls. */
typedef struct {
    int32_t nx, ny, nz; /* >= 1 each; the IB calls need nx, nz >= 4 */
    int32_t walls;      /* 1 = bounce-back walls normal to y (planes y = -1/2, ny - 1/2);
                           2 = on-site velocity walls on rows 0 and ny-1 (Eq. (23)-(30), turned
                           to a y-normal wall; ny >= 3): the populations entering a wall row
                           are set so that its velocity (sum c f + F/2)/rho equals the wall's,
                           i.e. the imposed momentum is rho u_w - F/2; 0 = periodic in y.
                           lbm_restrict and closure_targets reject 2 (LBM_ERR_UNSUPPORTED). */
    float tau;          /* > 0.5 */
    float body_force[3];
    float u_wall_lo[3]; /* velocity of the lower wall (y = -1/2; row 0 on-site); y component 0 */
    float u_wall_hi[3]; /* velocity of the upper wall (y = ny - 1/2; row ny-1 on-site); y component 0 */
} lbm_params;

/* Bytes of device workspace for `nch` channels with the given storage and room for up to
 * `max_nodes` immersed-boundary nodes in total (0: no IB).  0 on invalid arguments. */
size_t lbm_workspace_bytes(const lbm_params* ch /*host [nch]*/, int32_t nch, lbm_storage storage,
                           int64_t max_nodes);

/* Create a context over a caller-owned device workspace (256-byte aligned, at least
 * lbm_workspace_bytes() bytes).  Enqueues the clearing of the workspace on `stream`.
 * The populations are undefined until lbm_init() or lbm_set_populations(). */
lbm_status lbm_create(const lbm_params* ch /*host [nch]*/, int32_t nch, lbm_storage storage,
                      ib_kernel kernel, int64_t max_nodes, void* workspace, size_t bytes, void* stream,
                      lbm_ctx** out /*host*/);

/* Synchronise the stream, release the handle (and any captured graph).  NULL is a no-op. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* f(x, 0) = f^eq(rho, u) of Eq. (20) at every cell.  rho: [cells] or NULL (rho = 1);
 * u: [3][cells] per channel or NULL, meaning the steady wall-driven profile
 * u(y) = u_lo + (u_hi - u_lo) (y + 1/2) / ny with walls, u_lo + (u_hi - u_lo) y / (ny - 1)
 * with on-site walls (zero without walls). */
lbm_status lbm_init(lbm_ctx* ctx, const float* rho, const float* u);

/* `nsteps` lattice-Boltzmann steps (section 3.3): collide with BGK (Eq. (16)) and the Guo
 * force term (Eq. (19), with the sign of the c_s^2 I term read as minus) using the force
 * F = body_force + g, g the field of the last ib_spread (zero if none), then stream with
 * halfway bounce-back (moving-wall term 6 w_i c_i.u_w) at the y-walls, or with the on-site
 * rule of Eq. (23)-(30) at the wall rows (walls = 2). */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Declare the Lagrangian nodes: n in total (<= max_nodes), node_offsets = host array of
 * nch+1 ascending offsets assigning nodes to channels (NULL allowed when nch == 1).
 * Must precede ib_spread / ib_interp. */
lbm_status ib_set_nodes(lbm_ctx* ctx, int64_t n, const int64_t* node_offsets /*host*/);

/* Eq. (34)-(35), h = 1: g(x) = sum_m F_m phi(x - X_m) phi(y - Y_m) phi(z - Z_m) over the
 * 4x4x4 stencil floor(X)-1 .. floor(X)+2 (x, z periodic; rows outside the walls dropped).
 * Replaces the previous force field; the field stays in effect for later lbm_step calls.
 * X: [3][n] float64, F: [3][n] float32.  Deterministic (fixed-point accumulation). */
lbm_status ib_spread(lbm_ctx* ctx, int64_t n, const double* X, const float* F);

/* Eq. (33), h = 1: U_m = sum_x v(x) phi phi phi over the same stencil, with the current
 * fluid velocity v = (sum_i c_i f_i + (body_force + g)/2) / rho (g: last spread field);
 * stencil rows inside a wall take that wall's velocity.  X: [3][n] float64 (normally the
 * positions given to the preceding ib_spread), U: [3][n] float32 output. */
lbm_status ib_interp(lbm_ctx* ctx, int64_t n, const double* X, float* U);

/* Position update after the interpolation (Fig. 1): X <- X + U (float64, dt = 1). */
lbm_status ib_advance(lbm_ctx* ctx, int64_t n, double* X, const float* U);

/* Eq. (17)-(18) and the velocity shift under Eq. (19) at every cell of the current state:
 * drho = rho - 1 = sum_i (f_i - w_i)  [cells] and v = (sum_i c_i f_i + (body_force + g)/2)
 * / rho  [3][cells] per channel.  Either pointer may be NULL. */
lbm_status lbm_moments(lbm_ctx* ctx, float* drho, float* v);

/* Current pre-collision populations f_i (not shifted), paper order, [19][cells] per
 * channel, float32.  lbm_set_populations takes the same layout and replaces the state.
 * With on-site walls the populations entering a wall row are those of the wall rule (with
 * the current force); lbm_set_populations ignores them there. */
lbm_status lbm_get_populations(lbm_ctx* ctx, float* f);
lbm_status lbm_set_populations(lbm_ctx* ctx, const float* f);

/* Raw state (the stored shifted post-collision buffer) for bit-exact checkpoint/resume:
 * lbm_state_bytes() bytes, device to device. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_get_state(lbm_ctx* ctx, void* dst);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* src);

/* Viscous stress of the Guo-forced BGK scheme at the wall-adjacent rows y = 0 (lo) and
 * y = ny-1 (hi): sigma_ab = -(1 - 1/2tau) sum_i c_ia c_ib (f_i - f_i^eq)
 * - (1 - 1/2tau)(F_a v_b + F_b v_a)/2 for (a,b) = (x,y) and (z,y); output [2][nz][nx]
 * per channel, concatenated.  (The paper gives no stress formula.) */
lbm_status lbm_wall_stress(lbm_ctx* ctx, float* lo, float* hi);

/* Synchronise the stream and return the OR of the device error bits since the last call
 * (LBM_FLAG_*), then clear them. */
lbm_status lbm_error_flags(lbm_ctx* ctx, uint32_t* flags /*host*/);

const char* lbm_status_string(lbm_status s);

/* ---------------------------------------------------------------- membrane forces
 * Forces on the Lagrangian nodes (Fig. 1, first box), the input of ib_spread:
 *   springs  Eq. (2)-(3): U = k/2 (|R| - L)^2 per edge, the force on a node is minus the
 *            gradient (a stretched edge pulls its ends together);
 *   bending  stand-in for Eq. (6)-(10): E = k_bend sum_hinges (1 - cos(theta - theta0)),
 *            theta the signed dihedral angle of the two triangles of a hinge;
 *   tethers  U = k_tether/2 |X - A|^2.
 * Connectivity is CSR so that every node gathers its own force (no atomics): a node evaluates
 * each hinge it belongs to for its own vertex.  All arrays are device memory; rest_len /
 * rest_cs are filled by ib_membrane_rest(). */
typedef struct {
    int64_t n;                 /* nodes */
    const int32_t* nbr_ptr;    /* [n+1] CSR over spring neighbours (both directions) */
    const int32_t* nbr_idx;    /* [nnz] neighbour node ids */
    double* rest_len;          /* [nnz] rest length per CSR entry */
    double k_spring;
    const int32_t* hinge_ptr;  /* [n+1] CSR node -> hinge incidences, or NULL */
    const int32_t* hinge_inc;  /* [nnz_h] (hinge id << 2) | role, role = slot 0..3 in the hinge */
    const int32_t* hinges;     /* [nh][4] (x0, x1, x2, x3): triangles (x0,x1,x2), (x3,x2,x1) */
    double* rest_cs;           /* [nh][2] cos and sin of the rest dihedral angle */
    int64_t nh;
    double k_bend;
    const double* anchors;     /* [3][n] tether anchors, or NULL */
    double k_tether;
    /* Area and volume constraints, Eq. (4)-(5), force -grad H: off when tri is NULL or the three
     * coefficients are 0.  Triangles (a, b, c) have the outward normal (b - a) x (c - a); each
     * body's triangles are contiguous.  Per body S^total and V are summed in a fixed order (one
     * workgroup per body), so the forces are deterministic. */
    const int32_t* tri;        /* [nt][3] */
    int64_t nt;
    const int32_t* tri_ptr;    /* [n+1] CSR node -> triangle incidences */
    const int32_t* tri_inc;    /* [nnz_t] (triangle id << 2) | corner 0..2 */
    const int32_t* tri_body;   /* [nt] body of each triangle */
    const int32_t* body_tri;   /* [nb+1] first triangle of each body, then nt */
    int64_t nb;
    double* rest_area;         /* [nt] S_0 of each triangle (filled by ib_membrane_rest) */
    double* rest_body;         /* [nb][2] S_0^total, V_0 of each body (filled by ib_membrane_rest) */
    double* body_now;          /* [nb][4] scratch: S^total, V of the current shape and the force
                                  coefficients k_s (S^total - S_0^total)/S_0^total, k_v (V - V_0)/V_0 */
    double k_area_global;      /* k_s of Eq. (4) */
    double k_area_local;       /* k_t of Eq. (4) */
    double k_volume;           /* k_v of Eq. (5) */
    /* Finite-element bending of Eq. (6)-(10) (section 3.1): off when elem6 is NULL or k_fe is 0.
     * Six-node quadratic triangles (Eq. (7)): corners a, b, c with outward normal
     * (b - a) x (c - a), then the midpoint nodes of a-b, b-c, c-a.  At every node of every
     * element the curvature tensor kappa of the interpolated surface solves Eq. (9), with the
     * surface normal n and the node's share of the area (a third of each of the element's four
     * flat sub-triangles around it); averaged over the node's elements they give the mean
     * curvature K = tr(kappa)/2 (Eq. (10)), the Gaussian curvature G = ((tr kappa)^2 -
     * tr(kappa kappa))/2, the unit normal and the area A.  Lap K is the node average of the
     * surface divergence of the node-averaged surface gradient of K.  Force on a node:
     * (k_fe/2)(Lap K + 2K(K^2 - G)) n A, the variational derivative of Eq. (6) (the force
     * printed after Eq. (10) omits k_fe/2 and the Gaussian-curvature term).  FP64 arithmetic. */
    const int32_t* elem6;      /* [ne][6] node ids */
    int64_t ne;
    const int32_t* elem_ptr;   /* [n+1] CSR node -> element-node incidences (6 ne in total) */
    const int32_t* elem_inc;   /* [6 ne] (element id << 3) | local node 0..5 */
    int32_t* elem_slot;        /* [ne][6] scratch: position of (element, local node) in elem_inc
                                  (set by ib_membrane_rest) */
    double* fe_work;           /* [84 ne + 6 n] scratch */
    double k_fe;               /* k_0 of Eq. (6) */
    /* Adhesion to the lower wall, section 3.2 (Eq. (12)-(14)): off when adh_nr is 0.  Receptor
     * point r lies in the triangle rec_tri[r] at barycentric weights rec_bary[r]; ligands are
     * points (x, z) on the wall plane y = adh_wall_y (x, z periodic with periods adh_nx, adh_nz).
     * A bond joins one receptor to one ligand (at most one per receptor, four per ligand) and
     * pulls as a spring of rest length adh_lb: F = -adh_sigma (|d| - adh_lb) d / |d|, d = receptor
     * - ligand, shared among the triangle's nodes by the weights; ib_membrane_forces adds it
     * (the H_wall term of Eq. (11)).  ib_adhesion_step (and every coupled step, after the move)
     * runs one Monte-Carlo step: bonds present at the start break with P_r = 1 - exp(-k_off),
     * k_off = adh_koff0 exp(adh_gamma F_b / adh_kT), F_b = adh_sigma | |d| - adh_lb | (Eq. (12));
     * receptors unbound at the start bid with P_f = 1 - exp(-k_on), k_on = adh_kon0
     * exp(adh_sigma s (adh_gamma - s/2) / adh_kT), s = | |d| - adh_lb | (Eq. (13) as printed), for
     * the nearest ligand (lower id on a tie) closer than adh_capture that had fewer than four
     * bonds at the start; each ligand accepts bids in ascending receptor id up to four bonds.
     * Rates are per step (rate times dt).  Uniforms: Philox4x32-10, key adh_seed, counter
     * (receptor, step, 0) with the step counted on the device from 0 (reset by ib_membrane_rest);
     * words 0-1 decide the break, 2-3 the bid, as (w0 >> 5) 2^-27 + (w1 >> 6) 2^-53.  FP64. */
    int64_t adh_nr;
    const int32_t* rec_tri;    /* [nr][3] node ids */
    const double* rec_bary;    /* [nr][3] barycentric weights */
    const int32_t* rec_ptr;    /* [n+1] CSR node -> receptor incidences (3 nr in total) */
    const int32_t* rec_inc;    /* [3 nr] (receptor << 2) | corner 0..2 */
    int64_t adh_nl;            /* ligands */
    const double* lig_xz;      /* [nl][2] */
    int32_t* bond;             /* [nr] state: ligand id or -1 (the caller sets the initial bonds) */
    int32_t* lig_count;        /* [nl] state: bonds per ligand (consistent with bond) */
    int32_t* adh_work;         /* [ib_adhesion_work_ints()] scratch: the ligand table by wall
                                  cell (built by ib_membrane_rest), the step counter, per-ligand
                                  bids; word 2 counts bids lost to a full bid list (results then
                                  differ from the stated rule) */
    double adh_wall_y, adh_nx, adh_nz, adh_capture, adh_sigma, adh_lb, adh_gamma, adh_kT;
    double adh_kon0, adh_koff0;
    uint64_t adh_seed;
} ib_membrane;

#define ADH_MAX_BIDS 32 /* bids a ligand can receive in one step */
/* int32 words of ib_membrane::adh_work for nl ligands on an nx x nz wall and the capture radius:
 * 8 + nl (3 + ADH_MAX_BIDS) + 2 (cells + 1), cells = gx gz, gx = max(1, floor(nx / capture)) and gz
 * likewise (evaluated in double precision); 0 on invalid arguments. */
int64_t ib_adhesion_work_ints(int64_t nl, double nx, double nz, double capture);

/* Measure rest lengths, rest dihedral angles and (with triangles) the rest areas and volumes
 * on X_rest ([3][n] float64); build elem_slot, and the ligand table of the adhesion.  Requires
 * every element node's incidences in elem_ptr / elem_inc. */
lbm_status ib_membrane_rest(const ib_membrane* m /*host*/, const double* X_rest, void* stream);
/* F = -grad(E)(X), float64 arithmetic, float32 output [3][n]. */
lbm_status ib_membrane_forces(const ib_membrane* m /*host*/, const double* X, float* F, void* stream);
/* One Monte-Carlo step of the adhesion (section 3.2) at the positions X ([3][n] float64): updates
 * bond, lig_count and the step counter.  LBM_ERR_ARG without adhesion. */
lbm_status ib_adhesion_step(const ib_membrane* m /*host*/, const double* X, void* stream);

/* ---------------------------------------------------------------- coupled sequence
 * `nsteps` full steps of Fig. 1 on the context's stream: ib_membrane_forces(X) ->
 * ib_spread(X, F) -> lbm_step(1) -> ib_interp(X) -> X += U (-> ib_adhesion_step(X) when the
 * membrane has adhesion).  m may be NULL (F given,
 * kept constant).  X is updated in place; F and U hold the last step's values. */
lbm_status lbm_coupled_steps(lbm_ctx* ctx, const ib_membrane* m /*host*/, int32_t nsteps, double* X,
                             float* F, float* U);

/* Capture `nsteps` coupled steps (even, >= 2, a multiple of 2 lbm_launch.rebin) into a HIP
 * graph held by the context, then
 * replay it `repeats` times per lbm_graph_launch.  The captured pointers must stay valid.
 * The context's stream must not be the legacy default (NULL) stream: LBM_ERR_UNSUPPORTED.
 * The graph reads and writes the population buffer and IB tile set that were current at
 * capture; a replay leaves them current again.  lbm_graph_launch returns LBM_ERR_STATE
 * (and launches nothing) when other calls since the capture left a different buffer or
 * tile set current, or a different point in the binning cycle: an odd number of eager coupled
 * steps (with rebin > 1: a number that is not a multiple of 2 rebin), a lone lbm_step or
 * ib_spread, a change of the launch configuration. */
lbm_status lbm_graph_capture(lbm_ctx* ctx, const ib_membrane* m /*host*/, int32_t nsteps, double* X,
                             float* F, float* U);
lbm_status lbm_graph_launch(lbm_ctx* ctx, int32_t repeats);

/* ---------------------------------------------------------------- learned closure
 * An extension of the collision step (the paper has none): a small network corrects the
 * post-collision non-conserved moments of the forced BGK update of Eq. (16), (19), (20).
 *   m    = M_nc (f - f^eq(rho, v))  the 15 non-equilibrium moments of the pre-collision
 *          state in the orthonormal D3Q19 moment basis M (Gram-Schmidt of the monomials
 *          1, x, y, z, x^2, y^2, z^2, xy, xz, yz, x^2y, x^2z, y^2x, y^2z, z^2x, z^2y,
 *          x^2y^2, x^2z^2, y^2z^2 of the lattice velocities; M_nc = rows 4..18)
 *   raw  = (m, |F_IB|)              16 inputs; F_IB the spread force at the cell
 *   x    = (raw - in_mean) * in_scale, rounded to bfloat16
 *   y    = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3   (hidden activations bfloat16,
 *          float32 accumulation on the matrix cores)
 *   dm   = y[0:15] * out_scale[0:15]
 *   f*   = f*_BGK + M_nc^T dm  if dm is finite and |dm|_2 <= c_guard |m|_2, else f*_BGK
 *          (the node falls back to the plain step: LBM_FLAG_CLOSURE_FALLBACK, counted).
 * Mass and momentum are untouched (M_nc is orthogonal to 1 and c).
 * Parameters: float32, flat, in the order W1[16][64], b1[64], W2[64][64], b2[64],
 * W3[64][16], b3[16] (W[in][out]); norm: in_mean[16], in_scale[16], out_scale[16]. */
#define MLP_PARAMS 6288
#define MLP_NORM 48
#define MLP_PACKED_BYTES 23360 /* bf16 matrix-core fragments + biases + scaling */

/* Convert params / norm (device) into the packed form the kernels read (device,
 * MLP_PACKED_BYTES, caller-owned), on `stream`. */
lbm_status mlp_pack(const float* params, const float* norm, float c_guard, void* packed, void* stream);

/* Enable (packs params / norm into the context's workspace; the inputs may be freed once the
 * stream has passed this call) or disable (enable = 0, pointers ignored) the closure in every
 * later lbm_step / coupled step of the context. */
lbm_status lbm_set_closure(lbm_ctx* ctx, const float* params, const float* norm, float c_guard, int32_t enable);

/* Synchronise the stream; return the number of node updates that fell back to the plain
 * step since the last call, then reset it. */
lbm_status lbm_closure_guarded(lbm_ctx* ctx, uint64_t* count /*host*/);

/* Network only (no guard): dm[b][k] = y_k * out_scale_k for B samples of raw inputs
 * raw[B][16] (device), output dm[B][16] (device; lane 15 is the unused output). */
lbm_status mlp_forward(const void* packed, const float* raw, int64_t B, float* dm, void* stream);

/* Gradient of the training loss L = sum_b sum_{k<15} (y_bk - t_bk)^2 / (15 B), with
 * t = target / out_scale, with respect to the flat parameters (grad[MLP_PARAMS], device) and
 * the loss itself (loss[1], device, may be NULL).  Forward and backward run on the BF16
 * matrix cores (float32 accumulation, the backward signals rounded to bfloat16); partial
 * sums of every workgroup are reduced in a fixed order, so the result is reproducible bit
 * for bit.  work: mlp_grad_workspace_bytes(B) bytes of device scratch. */
size_t mlp_grad_workspace_bytes(int64_t B);
lbm_status mlp_grad(const void* packed, const float* raw, const float* target, int64_t B, float* grad,
                    float* loss, void* work, size_t work_bytes, void* stream);

/* mlp_grad for callers that cannot allocate device memory (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): the same kernels, the same partition of the
 * B samples over workgroups and so the same bits as mlp_grad, with the per-workgroup partial
 * sums in a scratch array the library holds per GPU (1024 rows of MLP_PARAMS + 1 floats,
 * 25.8 MB, kept until the process ends) instead of a caller workspace.  It calls no allocating
 * routine.  The scratch's address on the current device is looked up on the first call there;
 * `stream` must belong to the current device (else LBM_ERR_ARG).  B >= 1; every B fits, since
 * the kernel never runs more than 1024 workgroups (a B needing more rows than the scratch holds
 * is rejected with LBM_ERR_ARG).  All calls on one GPU share its scratch: calls that overlap in
 * time on that GPU (different streams, host threads) race and must be serialised by the caller;
 * calls in order on one stream are safe, and nothing needs clearing between them. */
lbm_status mlp_grad_noalloc(const void* packed, const float* raw, const float* target, int64_t B, float* grad,
                            float* loss, void* stream);

/* Adam (Kingma & Ba 2015) on n float32 parameters: m, v are the moment buffers (zero at
 * step 1), step counts from 1. */
lbm_status mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* stream);

/* Input / output scaling from B training samples: in_mean = mean(raw), in_scale =
 * 1/std(raw) (1 where std = 0), out_scale = rms(target) (1 where 0); norm[MLP_NORM] device.
 * work: mlp_norm_workspace_bytes(B) bytes of device scratch; fixed-order reduction. */
size_t mlp_norm_workspace_bytes(int64_t B);
lbm_status mlp_norm(const float* raw, const float* target, int64_t B, float* norm, void* work, size_t work_bytes,
                    void* stream);

/* Training data.  lbm_restrict: 2x restriction (acoustic scaling, dt_c = 2 dt_f) of the
 * current state of a one-channel fine context with even nx, ny, nz into coarse shifted
 * pre-collision populations g_c = f_c - w ([19][Nc], paper order, Nc = nx ny nz / 8):
 * rho_c and j_c are the 2x2x2 block means, f_c = f^eq(rho_c, j_c/rho_c) + (2 tau_c / tau_f)
 * * mean(f - f^eq(rho, j/rho)) (Dupuis & Chopard rescaling), and the coarse IB force
 * density F_c = 2 mean(F_IB) ([3][Nc]) from the fine context's latest spread.
 * closure_targets: for one coarse step from g0 (force body + F) to g1 (both shifted
 * pre-collision, [19][N]) on the coarse channel `coarse` (host): raw features feat[N][16]
 * of g0 and targets target[N][16] = (M_nc (unstream(g1) - collide(g0)), 0), where unstream
 * inverts the streaming and bounce-back of the coarse step exactly. */
lbm_status lbm_restrict(lbm_ctx* fine, float tau_coarse, float* g_c, float* F_c);
lbm_status closure_targets(const lbm_params* coarse /*host*/, const float* g0, const float* F, const float* g1,
                           float* feat, float* target, void* stream);

/* ---------------------------------------------------------------- launch tuning
 * Launch shape of the lattice kernel, chosen by the autotuner (defaults are valid). */
typedef struct {
    int32_t block;       /* threads per workgroup: 64, 128, 256, 512 or 1024 */
    int32_t xcd_remap;   /* 1 = map consecutive lattice segments to the same XCD */
    int32_t persistent;  /* 0 = one workgroup per segment; >0 = that many resident workgroups looping */
    int32_t nontemporal; /* 1 = non-temporal stores of the new populations */
    int32_t vec;         /* cells per lane: 0/1 scalar step; 2 or 4 = vector step (aligned V-wide
                            accesses, 256-thread workgroups), used when every channel has
                            nx % V == 0 and nx*ny*nz % (64 V) == 0, else the scalar step runs */
    int32_t overlap;     /* coupled steps only: 1 = the lattice update with the body force alone runs
                            on a second stream, overlapped with the previous interpolation and the
                            force / spread pipeline, then the cells of the flagged IB tiles are
                            updated again with their force (the same values as the fused update,
                            bit for bit); 0 = one fused update after the spread.  Ignored while
                            the learned closure is enabled.  Default 0: on MI355X the
                            bandwidth-bound update occupies every CU and the latency-bound IB
                            kernels beside it slow down more than the overlap gains. */
    int32_t split;       /* coupled steps without the closure or overlap: 1 = the lattice update with
                            the body force alone runs in the same launch as the spread, then the
                            flagged tiles' cells are updated with their force (merging split
                            tiles' partial sums on the way); 0 = spread, merge, one fused update;
                            -1 (default) = 1 for a single channel, 0 for several.  Bitwise the
                            same results.  It pays when the flagged tiles are a few percent of the
                            lattice (one channel with 16 platelets: 2.7%, 195 -> 190 us per step)
                            and loses when they are many (the 64-channel batch: 10%). */
    int32_t rebin;       /* coupled steps with a membrane: the nodes are binned into the IB tile
                            lists every `rebin` steps (1..64; 1 = every step, the default).  With
                            rebin > 1 a node is listed in every tile its stencil can reach while it
                            stays within half a lattice spacing of where it was binned; the steps
                            in between recompute only the nodes' stencil weights (in the force
                            kernel) and reuse the lists.  The spread sums exact integers over
                            the tiles' cells, so the results are bitwise those of rebin = 1; a node
                            that moves further sets LBM_FLAG_REBIN_MARGIN (its contributions to
                            unlisted tiles are lost).  A captured graph must then hold a multiple
                            of 2 rebin steps. */
} lbm_launch;

lbm_status lbm_set_launch(lbm_ctx* ctx, const lbm_launch* cfg /*host*/);
lbm_status lbm_get_launch(const lbm_ctx* ctx, lbm_launch* cfg /*host*/);

/* Measurement helper, not part of the method: with enable = 1 every later eager
 * lbm_coupled_steps call (not graph capture, not the overlapped schedule) records a pair of
 * timing events on the context's stream around the launch that updates the lattice: the
 * body-force update of every cell that also runs the spread (split schedule, kind 1), the
 * fused lattice step (kind 0) or the closure step (kind 2); at most LBM_TIMER_PAIRS launches
 * are timed.  lbm_launch_timer_read synchronises the stream, returns the number of timed
 * launches, their mean duration in microseconds and the kind of the last one (kind may be
 * NULL), and starts a new count.  Enabling again resets the count. */
#define LBM_TIMER_PAIRS 1024
lbm_status lbm_launch_timer(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_launch_timer_read(lbm_ctx* ctx, int64_t* count /*host*/, double* mean_us /*host*/,
                                 int32_t* kind /*host*/);

/* Measurement helper, not part of the method: copy `bytes` (multiple of 16) from src to dst
 * with 16-byte accesses (variant 0: plain stores, 1: non-temporal stores), `grid`
 * workgroups of 256 threads (0: one 16-byte element per thread).  Gives the practical HBM
 * ceiling a lattice step is compared with. */
lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, int32_t variant, int64_t grid, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MI355_LBMIB_H */
