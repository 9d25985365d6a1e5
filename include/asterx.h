/* asterx.h -- C ABI of the MI355X (gfx950) library for the Valencia GRMHD right-hand side
 * of AsterX (arXiv 2406.11669) on one 3-D Cartesian block with a given 3+1 metric.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument is a DEVICE pointer owned by the caller unless it is
 *   documented as host memory.  The library keeps no pointer after a call returns and
 *   never allocates or frees memory in these calls.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *   calls are asynchronous on it; none synchronizes the device.
 * Errors.  Return 0 on success.  A negative value means an argument error detected on the
 *   host before anything was launched (ASTERX_EARG) or a launch failure (ASTERX_ELAUNCH);
 *   asterx_last_error() then returns a message (thread-local, valid until the next call).
 *   Physical failures of the primitive recovery are not errors: they are counted in the
 *   device-side statistics and per-cell flags.
 * Layout (paper Sec. 3.1, storage locations).  All fields of a block share one padded
 *   index space of extents ld[0] x ld[1] x ld[2], x fastest; field f of a multi-field
 *   array starts at f * ld[0]*ld[1]*ld[2].  Index (i,j,k), i in [-ng, n+ng], is stored at
 *   ((k+ng)*ld[1] + (j+ng))*ld[0] + (i+ng) and names: the cell centre (i,j,k); the x-face
 *   (i-1/2,j,k), y-face (i,j-1/2,k), z-face (i,j,k-1/2); the x-edge (i,j-1/2,k-1/2),
 *   y-edge (i-1/2,j,k-1/2), z-edge (i-1/2,j-1/2,k); the vertex (i-1/2,j-1/2,k-1/2).
 *   Owned indices are 0..n-1 per axis; all others are ghosts, filled by the caller (or
 *   asterx_fill_ghosts) before they are read.
 * Field orders.
 *   metric [10] at vertices: alpha, beta^x, beta^y, beta^z, g_xx, g_xy, g_xz, g_yy, g_yz, g_zz
 *   curv   [6]  at vertices: K_xx, K_xy, K_xz, K_yy, K_yz, K_zz (extrinsic curvature)
 *   prim   [5]  at centres : rho, p, v^x, v^y, v^z (Eulerian 3-velocity, contravariant)
 *   cons   [5]  at centres : sqrt(gamma) (D, S_x, S_y, S_z, tau) (densitized, Sec. 2.2)
 *   A      [3]  at edges   : A_x, A_y, A_z (vector potential, Sec. 2.3)
 *   psi    [1]  at vertices: Psi_mhd = sqrt(gamma) Phi (Sec. 3.4)
 *   state / rhs [9]        : cons (5), A (3), psi (1) in that order
 */
#ifndef ASTERX_H
#define ASTERX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASTERX_OK 0
#define ASTERX_EARG (-1)
#define ASTERX_ELAUNCH (-2)

enum { ASTERX_RECON_MINMOD = 0, ASTERX_RECON_PPM = 1, ASTERX_RECON_WENOZ = 2, ASTERX_RECON_MP5 = 3 };
enum { ASTERX_RIEMANN_HLLE = 0, ASTERX_RIEMANN_LXF = 1 };
enum { ASTERX_CT_FCT = 0, ASTERX_CT_UCT = 1 };
enum { ASTERX_GAUGE_LORENZ = 0, ASTERX_GAUGE_ALGEBRAIC = 1 };
enum { ASTERX_SPEEDS_QUARTIC = 0, ASTERX_SPEEDS_BOUND = 1 };
enum { ASTERX_C2P_NOBLE_PALENZUELA = 0, ASTERX_C2P_NOBLE_ONLY = 1, ASTERX_C2P_PALENZUELA_ONLY = 2 };
enum { ASTERX_BC_PERIODIC = 0, ASTERX_BC_COPY = 1, ASTERX_BC_LINEAR = 2 };

/* per-cell c2p flag bits */
enum {
  ASTERX_FLAG_NOBLE_FAIL = 1, ASTERX_FLAG_FALLBACK = 2, ASTERX_FLAG_ATMOSPHERE = 4,
  ASTERX_FLAG_HARD_FAIL = 8, ASTERX_FLAG_NAN_IN = 16
};

/* Block geometry.  n: owned cells per axis (>= 1); ng: ghost layers (>= 3 for
 * asterx_rhs, whose face stencils span six cells; >= 2 elsewhere); ld: allocated extents
 * (>= n + 2 ng + 1; ld[0]*ld[1]*ld[2] below 2^29, so that byte offsets within a field fit 32 bits); dx: spacing. */
typedef struct {
  int32_t n[3];
  int32_t ng;
  int32_t ld[3];
  int32_t pad_;
  double dx[3];
} asterx_grid;

/* Method parameters (paper Secs. 3.3-3.7). */
typedef struct {
  double gamma;     /* ideal-gas adiabatic index (Sec. 3.7), > 1 */
  double rho_atm;   /* atmosphere density floor (Sec. 3.6), >= 0 */
  double k_atm;     /* polytropic constant of the atmosphere pressure p = K rho^Gamma */
  double xi;        /* generalized-Lorenz damping in units of 1/dt_max (Sec. 3.4: 1.5) */
  double c2p_tol;   /* Noble Newton tolerance on max(|dz/z|, |dw|) */
  double wmax;      /* Lorentz-factor safety cap of the c2p clamps (> 1) */
  double weno_eps;  /* WENO-Z epsilon */
  double weno_q;    /* WENO-Z exponent (1 or 2) */
  int32_t c2p_maxit;   /* Noble iteration cap */
  int32_t brent_maxit; /* Brent iteration cap */
  int32_t recon;       /* ASTERX_RECON_* */
  int32_t gauge;       /* ASTERX_GAUGE_* */
  int32_t speeds;      /* ASTERX_SPEEDS_* */
  int32_t c2p_method;  /* ASTERX_C2P_* */
  int32_t riemann;     /* ASTERX_RIEMANN_*: HLLE (Sec. 3.3 eq. HLLEfluxes) or Lax-Friedrichs (eq. LxFfluxes) */
  int32_t ct;          /* ASTERX_CT_*: edge electric field by flux CT (averaged face induction fluxes) or
                          upwind CT (Sec. 3.4, eqs. uct1, uct2, eq3.20: upwind face velocities and face
                          fields reconstructed to the edges by PPM).  Upwind CT needs ng >= 4, is for
                          single blocks (asterx_rhs, asterx_rhs_rk; the batch calls refuse it) and is
                          not differentiated (asterx_rhs_adjoint refuses it). */
} asterx_params;

/* Device-side counters, accumulated (never reset) by asterx_c2p. */
typedef struct {
  unsigned long long noble_fail, fallback_used, atmosphere, hard_fail, nan_in, iters_max;
} asterx_c2p_stats;

int asterx_version(void);
const char* asterx_last_error(void);

/* Bytes of device workspace asterx_rhs needs for this grid. */
size_t asterx_rhs_workspace_size(const asterx_grid* g);

/* Primitive -> conserved map on owned cells (Sec. 2.2, conserved-variable definitions;
 * Sec. 3.12: analytic initialisation of the conserved variables).  Reads metric at
 * vertices i-1..i+2 (4th-order interpolation to the centre, Sec. 3.2) and A around the
 * cell (centre field = average of the two faces of the curl, Sec. 3.1).  Writes cons on
 * owned cells only. */
int asterx_prim2con(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A,
                    const double* prim, double* cons, void* stream);

/* Conservative-to-primitive recovery on owned cells (Sec. 3.5): Noble et al. 2D Newton in
 * (z = rho h W^2, w = v^2) warm-started from `prim`, Palenzuela et al. 1D Brent fallback in
 * x = h W, atmosphere (Sec. 3.6) when D < sqrt(gamma) rho_atm, when rho < rho_atm after
 * recovery, or when both solvers fail.  In/out: cons (reset to the atmosphere state where
 * applied), prim (guess in, result out).  flags: u8 per point (may be NULL).  stats:
 * device asterx_c2p_stats (may be NULL), accumulated. */
int asterx_c2p(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A,
               double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream);

/* Ghost fill of nf consecutive fields of f, axis by axis (x, then y, then z) over the full
 * extent of the other axes, so edges and corners are filled.  kinds: host int[3], one
 * ASTERX_BC_* per axis.  PERIODIC: index s maps to s mod n; COPY: nearest owned index;
 * LINEAR: linear extrapolation from the two nearest owned indices. */
int asterx_fill_ghosts(const asterx_grid* g, double* f, int32_t nf, const int32_t* kinds, void* stream);

/* Periodic ghost fill of nf <= 3 fields with a constant added per period of wrap:
 * f(s) = f(s mod n) + shift[q*3 + d] * floor(s / n) for field q along axis d.  This is the
 * periodic image of a vector potential A = B_mean x r / 2 + (periodic part) of a field with
 * a uniform mean.  shift: host double[nf*3]. */
int asterx_fill_ghosts_shift(const asterx_grid* g, double* f, int32_t nf, const double* shift, void* stream);

/* Right-hand side of the 9 evolved fields on owned points (Sec. 2.2 eq. fluxconseqs and
 * grmhdsrc; Sec. 3.3 reconstruction + HLLE; Sec. 3.4 FCT electric field, gauge terms and
 * the Psi equation; Sec. 3.12 workflow).  Reads prim on ng ghost layers, A on ng layers,
 * psi and metric/curv on 2 layers.  dt_max sets xi = p->xi / dt_max.  red: device
 * double[2] updated with max(red, value): [0] max characteristic speed over the faces of
 * owned cells, [1] max |div Btilde| over owned cells (may be NULL).  workspace: device
 * buffer of at least asterx_rhs_workspace_size(g) bytes. */
int asterx_rhs(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
               const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
               void* workspace, size_t ws_bytes, void* stream);

/* Runge-Kutta stage combine on owned points of the 9 state fields (the RK4 and RK2 time
 * integrators of the tests and benchmarks, Sec. 4 and 5):
 * out = sum_m a[m] u[m] + b_dt rhs.  a: host double[nterms]; u: host array of nterms
 * device pointers (each a 9-field state); 1 <= nterms <= 4; out may alias any u[m]. */
int asterx_rk_stage(const asterx_grid* g, int32_t nterms, const double* a, const double* const* u, double b_dt,
                    const double* rhs, double* out, void* stream);

/* One Runge-Kutta stage output of asterx_rhs_rk: out = sum_m a[m] u[m] + b_dt rhs on owned
 * points of the 9 state fields, rhs being the right-hand side the call evaluates.  u: nterms
 * (1 or 2) device 9-field states; out: device 9-field state. */
typedef struct {
  int32_t nterms;
  double a[2];
  const double* u[2];
  double b_dt;
  double* out;
} asterx_rk_out;

/* asterx_rhs followed by asterx_rk_stage for each of nout (1 or 2) outputs, without storing
 * the right-hand side: the cell and edge kernels combine each point's value into the outputs
 * as they produce it (the Runge-Kutta stage update of Sec. 4 and 5), with the same
 * arithmetic as asterx_rk_stage, so the results agree bit for bit.  outs: host
 * asterx_rk_out[nout].  An output may be one of its own states u[m] (updated in place) but
 * must not overlap the other output or the states it reads, nor metric, curv, prim, A, psi
 * or the workspace: the state whose right-hand side is evaluated is read by neighbouring
 * points while outputs are written (ASTERX_EARG otherwise).  Other arguments as asterx_rhs. */
int asterx_rhs_rk(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
                  const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                  const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream);

/* asterx_rhs_rk without a caller-provided workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * workspace is a library-held device array of ASTERX_NOALLOC_WS_BYTES (64 MiB) per device,
 * enough for blocks whose asterx_rhs_workspace_size is at most that (cubes up to 52^3 cells
 * with 3 ghost layers; ASTERX_EARG beyond, before any launch).  The call allocates and frees nothing.
 * The array used is the one of the device current on the calling thread, which must be the
 * device of `stream`.  Every call on a device shares that device's array and nothing in it
 * needs to start at zero (each call writes all it reads); calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller.  Other arguments,
 * results and errors as asterx_rhs_rk. */
#define ASTERX_NOALLOC_WS_BYTES (64ull << 20)
int asterx_rhs_rk_noalloc(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
                          const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                          const asterx_rk_out* outs, double* red, void* stream);

/* Covariant stress-energy tensor T_{mu nu} (eq. tmunu, lowered with the 4-metric) at the vertices
 * [0, n]^3 of the block, where Sec. 3.1 stores it with the spacetime variables for a spacetime
 * solver.  The vertex fluid state is the mean of the primitives (prim) and of the centre fields
 * (from the curl of A) of the 8 cells sharing the vertex; the metric is the vertex's own (metric).
 * Reads prim on one ghost layer and A on two.  tmunu: device, 10 vertex fields T_00, T_0x, T_0y,
 * T_0z, T_xx, T_xy, T_xz, T_yy, T_yz, T_zz in the block's layout; other points are not written. */
int asterx_tmunu(const asterx_grid* g, const asterx_params* p, const double* metric, const double* prim,
                 const double* A, double* tmunu, void* stream);

/* ---- Factor-2 mesh refinement: inter-level operators --------------------------------------
 * For refinement boundaries (Sec. 3.9; the prolongation of the AMR tests of Sec. 4): the fine
 * grid's vertex 0 sits on coarse vertex c0 (host int[3], coarse indices), fine spacing = coarse / 2.
 * stag (host int[3]): per axis, 0 if the field is cell-centred along it, 1 if vertex-centred
 * (conserved variables 0,0,0; metric and Psi 1,1,1; A_x 0,1,1; A_y 1,0,1; A_z 1,1,0).  nf fields
 * with the grids' field strides.  Other points of the target are not written.
 * asterx_prolong fills fine points lo..hi (host int[3], fine indices, inclusive; ghosts allowed):
 * vertex directions inject on coincident points and take the cubic Lagrange midpoint value
 * (-1, 9, 9, -1)/16 in between; cell directions give the two children of coarse cell c the
 * conservative third-order values u_c -+ (u_{c+1} - u_{c-1})/8; tensor product.  Fields centred in
 * all directions fall back, per coarse cell, to minmod-limited linear children when a third-order
 * child would leave [min, max] of the 27 coarse cells around the parent (the shock fallback; one
 * decision per parent keeps the children's mean equal to the parent).
 * asterx_restrict fills coarse points lo..hi (coarse indices): the mean of the children along
 * cell directions, injection along vertex directions; restriction undoes prolongation.
 * ASTERX_EARG when a box or the stencil it reaches leaves the stored points of either grid. */
int asterx_prolong(const asterx_grid* coarse, const asterx_grid* fine, const int32_t* c0, const int32_t* stag,
                   int32_t nf, const double* cf, double* ff, const int32_t* lo, const int32_t* hi, void* stream);
int asterx_restrict(const asterx_grid* coarse, const asterx_grid* fine, const int32_t* c0, const int32_t* stag,
                    int32_t nf, const double* ff, double* cf, const int32_t* lo, const int32_t* hi, void* stream);

/* Sets red[0..1] to 0 (device double[2]); a kernel, not a memset, so that it can be
 * recorded in a captured graph. */
int asterx_zero(double* buf, int64_t count, void* stream);

/* ---- Batches of patches ----------------------------------------------------------------
 * Many blocks ("patches", e.g. the boxes of a mesh-refinement hierarchy, each with its own
 * n, ld and dx) advanced together: every phase is one launch of a persistent grid whose
 * workgroups walk a precomputed list of (patch, tile) work items, instead of one launch per
 * patch.  Arrays of a batch are field-major pools: field f of patch p starts at
 * f * asterx_batch_points(b) + asterx_batch_offset(b, p) and uses the patch's own padded
 * index space from there (the single-block layout with the pool's field stride).  The
 * batch calls have the single-block semantics on every patch. */
typedef struct asterx_batch asterx_batch;

/* Schedule of the persistent launches: workgroups per compute unit, and the order of the
 * work list (0: patches as given; 1: largest patch first; 2: round robin over patches,
 * largest first). */
typedef struct {
  int32_t blocks_per_cu;
  int32_t order;
} asterx_batch_tuning;

/* Creates the work lists (host memory, plus small device tables it allocates and
 * asterx_batch_destroy frees; the only allocating calls of the library).  grids: host
 * array of npatches descriptors (ng >= 3 each); tuning may be NULL (4 per CU, order 1). */
int asterx_batch_create(int32_t npatches, const asterx_grid* grids, const asterx_batch_tuning* tuning,
                        asterx_batch** out);
int asterx_batch_destroy(asterx_batch* b);
int64_t asterx_batch_points(const asterx_batch* b);
int64_t asterx_batch_offset(const asterx_batch* b, int32_t p);
size_t asterx_batch_workspace_size(const asterx_batch* b);
int asterx_batch_prim2con(const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
                          const double* prim, double* cons, void* stream);
int asterx_batch_c2p(const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
                     double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream);
int asterx_batch_fill_ghosts(const asterx_batch* b, double* f, int32_t nf, const int32_t* kinds, void* stream);
int asterx_batch_rhs(const asterx_batch* b, const asterx_params* p, const double* metric, const double* curv,
                     const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
                     void* workspace, size_t ws_bytes, void* stream);
int asterx_batch_rk_stage(const asterx_batch* b, int32_t nterms, const double* a, const double* const* u,
                          double b_dt, const double* rhs, double* out, void* stream);
int asterx_batch_rhs_rk(const asterx_batch* b, const asterx_params* p, const double* metric, const double* curv,
                        const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                        const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream);

/* ---- Adjoint (reverse mode) ---------------------------------------------------------------
 * Vector-Jacobian products for differentiating whole RK steps with respect to the state and
 * the adiabatic index.  Periodic blocks only (every axis; n > ng): the transposed ghost fill
 * is the periodic one.  The forward maps are evaluated again inside these calls (c2p warm-
 * started from prim_guess); inputs are not modified.  Cotangent outputs are ACCUMULATED
 * (+=) on owned points; gamma_bar is a device double[1], accumulated.  Non-smooth points
 * take the active branch (an exact tie of the two HLLE sides splits evenly); converged
 * iterations are differentiated implicitly.  workspace: asterx_adjoint_workspace_size. */
size_t asterx_adjoint_workspace_size(const asterx_grid* g);

/* L(U) = rhs(fill(c2p(cons, A)), A, psi) (the right-hand side of asterx_rhs with the c2p that
 * precedes it in a stage).  Given rhs_bar (9 fields, owned points), adds L^T rhs_bar to
 * cons_bar (5), A_bar (3), psi_bar (1) and gamma_bar. */
int asterx_rhs_adjoint(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
                       const double* cons, const double* prim_guess, const double* A, const double* psi,
                       double dt_max, const double* rhs_bar, double* cons_bar, double* A_bar, double* psi_bar,
                       double* gamma_bar, void* workspace, size_t ws_bytes, void* stream);

/* prim = c2p(cons, A): given prim_bar (5 fields, owned), adds to cons_bar, A_bar, gamma_bar. */
int asterx_c2p_adjoint(const asterx_grid* g, const asterx_params* p, const double* metric, const double* cons,
                       const double* prim_guess, const double* A, const double* prim_bar, double* cons_bar,
                       double* A_bar, double* gamma_bar, void* workspace, size_t ws_bytes, void* stream);

/* cons = prim2con(prim, A): given cons_bar (5 fields, owned), adds to prim_bar, A_bar, gamma_bar. */
int asterx_prim2con_adjoint(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A,
                            const double* prim, const double* cons_bar, double* prim_bar, double* A_bar,
                            double* gamma_bar, void* workspace, size_t ws_bytes, void* stream);

/* ---- Independent points and the learned c2p initial guess ---------------------------------
 * Flat arrays of n points, field-major ([q * n + i]): metric 10 x n (alpha, beta^i, gamma_ij),
 * Btilde 3 x n (densitized), prim 5 x n, cons 5 x n (densitized).  gam_pts: per-point adiabatic
 * index (n doubles) or NULL for the scalar gam.  All arrays are device memory. */

/* cons = prim2con(prim) per point (eqs. of the conserved variables, Sec. 2.2).  target (2 x n,
 * optional): log W and log(z / D) with z = rho h W^2, the quantities the network predicts. */
int asterx_prim2con_points(int64_t n, const double* gam_pts, double gam, const double* metric, const double* Bt,
                           const double* prim, double* cons, double* target, void* stream);

/* Multilayer perceptron 8 -> 64 -> 64 -> 2, ReLU hidden activations, packed FP32 parameters
 * (device, ASTERX_MLP_NPARAMS floats): W1[64][8], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
 * Inputs are standardised as (f - in_shift) * in_scale; outputs are out_shift + out_scale * y.
 * Contractions run on bfloat16 operands with FP32 accumulation (matrix cores). */
#define ASTERX_MLP_NPARAMS 4866
typedef struct {
  const float* params;
  float in_shift[8], in_scale[8];
  float out_shift[2], out_scale[2];
} asterx_mlp;

/* The network's raw input features of conserved states (8 x n floats): log D, log(tau/D),
 * log(1 + S^2/D^2), log(1 + B^2/D), log(1 + (B.S)^2/D^3), det(gamma) - 1, alpha - 1, Gamma, with
 * D, S, tau, B undensitized.  States with D <= 0 or tau <= 0 give zeros. */
int asterx_mlp_features(int64_t n, const double* gam_pts, double gam, const double* metric, const double* Bt,
                        const double* cons, float* feat, void* stream);

/* out (2 x n floats) = network outputs (log W, log(z / D)) of the raw features feat (8 x n). */
int asterx_mlp_forward(const asterx_mlp* m, int64_t n, const float* feat, float* out, void* stream);

/* Loss (1/n) sum_i |y_i - t_i|^2 / 2 on standardised outputs (t = (target - out_shift) / out_scale)
 * and its gradient: grad[0..NPARAMS) = d loss / d params, grad[NPARAMS] = loss (device floats,
 * overwritten).  Deterministic (fixed-order reductions).  workspace: asterx_mlp_grad_workspace_size. */
size_t asterx_mlp_grad_workspace_size(int64_t n);
int asterx_mlp_grad(const asterx_mlp* m, int64_t n, const float* feat, const float* target, float* grad,
                    void* workspace, size_t ws_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) on the ASTERX_MLP_NPARAMS FP32 parameters; m, v are
 * the first and second moment buffers (device, zero before step 1). */
int asterx_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                    float eps, int32_t step, void* stream);

/* c2p of independent points (Sec. 3.5 and 3.6), in place on cons for atmosphere resets.  Initial
 * guess for Noble's iteration: the network's (W, z) when mlp is non-NULL (falling back to the
 * plain start if it does not converge, flag 32), else the primitives guess (5 x n, NULL: cold
 * start from the conserved variables).  flags (n bytes), iters (n int32) optional.  stats
 * (optional, 7 counters, accumulated): Noble failures, fallbacks, atmosphere, hard failures,
 * NaN inputs, max iterations (max), learned guesses not converged. */
int asterx_c2p_points(const asterx_params* p, int64_t n, const double* gam_pts, const double* metric,
                      const double* Bt, double* cons, const double* guess, const asterx_mlp* mlp, double* prim,
                      uint8_t* flags, int32_t* iters, unsigned long long* stats, void* stream);

/* asterx_c2p with the learned guess: each cell's Noble iteration starts from the network's
 * (W, z) (Sec. 3.5 solver unchanged); if that start does not converge, flag 32 is set and
 * the warm start from prim (cold start if unusable), Palenzuela and the atmosphere follow as
 * in asterx_c2p.  Cells below the density floor or with non-finite input skip the network.
 * Arguments as asterx_c2p, plus the network (see asterx_mlp). */
int asterx_c2p_learned(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A,
                       double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, const asterx_mlp* mlp,
                       void* stream);

/* ---- One stage with the recovery and the sources together -------------------------------
 * The geometric sources of the right-hand side (Sec. 2.2, eq. grmhdsrc) at a cell depend only
 * on the cell's primitives, its centre field and the centre metric with its derivatives and the
 * extrinsic curvature.  asterx_c2p_src recovers the primitives (asterx_c2p, or asterx_c2p_learned
 * when mlp is not NULL) and then evaluates these sources from the recovered state in the same
 * kernel, whose centre-metric values serve both; asterx_rhs_rk_src is asterx_rhs_rk with the
 * sources taken from there.  The pair gives bitwise the results of asterx_c2p (or
 * asterx_c2p_learned) followed by asterx_rhs_rk.
 * c2p_src: curv is K_ij at vertices ([6], as in asterx_rhs); src (device, ASTERX_SRC_FIELDS
 * fields of the block's index space, out): fields 0-3 receive alpha sqrt(gamma) times the sources
 * of S_x, S_y, S_z and tau on owned cells (that of D is 0); fields 4-13 the ten metric components
 * at the x faces of owned cells (Sec. 3.2 interpolation, indexed like cells: the face between
 * cells i-1 and i at cell i, i = 0..n), which the kernel's centre-derivative passes form on the
 * way.  Other arguments as asterx_c2p.  rhs_rk_src: src as written by asterx_c2p_src for the same
 * prim, A and metric (the x faces read their metric from it); other arguments as asterx_rhs_rk
 * (the outputs may not overlap src either). */
#define ASTERX_SRC_FIELDS 14
int asterx_c2p_src(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
                   const double* A, double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats,
                   const asterx_mlp* mlp, double* src, void* stream);
int asterx_rhs_rk_src(const asterx_grid* g, const asterx_params* p, const double* metric, const double* prim,
                      const double* A, const double* psi, const double* src, double dt_max, int32_t nout,
                      const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream);

/* Per-kernel timing (diagnostics).  When enabled, every launch of the library is bracketed
 * by two HIP events on its stream; asterx_timing_read waits for the recorded events and
 * returns, for each kernel class k < n, the accumulated milliseconds ms[k] and launch count
 * counts[k] (either may be NULL); it returns the number of kernel classes.
 * asterx_timing_name(k) names class k.  Do not enable while a stream is being captured.  The
 * timing state is process-global and unsynchronized: enable it only while one host thread
 * drives the library (the other entry points keep no host state across calls, except
 * asterx_last_error, which is per thread, and the no-allocation entry point's per-device
 * address table, which is locked). */
int asterx_timing_enable(int32_t on);
int asterx_timing_read(double* ms, long long* counts, int32_t n);
int asterx_timing_reset(void);
const char* asterx_timing_name(int32_t k);

#ifdef __cplusplus
}
#endif
#endif /* ASTERX_H */
