/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q19 / D3Q27 lattice Boltzmann
 * library.
 *
 * Method: Bauer & Ruede, "An improved lattice Boltzmann D3Q19 method based on
 * an alternative equilibrium discretization" (arXiv:1803.04937).
 *
 * One library call = one or more HIP kernel launches on the caller's stream.
 * All big buffers (PDF states, adjoint fields, checkpoints, moment fields,
 * link words) are caller-owned device memory; the library only allocates a
 * few small scratch buffers (reduction partials) per context.  Pointers are borrowed
 * and must outlive the context.  No function throws across the ABI: each
 * returns an lbm_status and lbm_last_error() gives the message.  A context
 * is not thread-safe; several contexts may coexist.  Every call is
 * stream-ordered and asynchronous except those that return values in host
 * memory (they synchronise the stream).
 *
 * Lattice (Sec. 2.3): D3Q19, directions in this fixed order, opposite
 * directions adjacent (opposite(q) = q + 1 for odd q, q - 1 for even q > 0):
 *    0 ( 0, 0, 0)
 *    1 ( 1, 0, 0)   2 (-1, 0, 0)   3 ( 0, 1, 0)   4 ( 0,-1, 0)
 *    5 ( 0, 0, 1)   6 ( 0, 0,-1)
 *    7 ( 1, 1, 0)   8 (-1,-1, 0)   9 ( 1,-1, 0)  10 (-1, 1, 0)
 *   11 ( 1, 0, 1)  12 (-1, 0,-1)  13 ( 1, 0,-1)  14 (-1, 0, 1)
 *   15 ( 0, 1, 1)  16 ( 0,-1,-1)  17 ( 0, 1,-1)  18 ( 0,-1, 1)
 * with weights 1/3 (rest), 1/18 (axis), 1/36 (edge).  D3Q27 appends the
 * eight corners
 *   19 ( 1, 1, 1)  20 (-1,-1,-1)  21 ( 1, 1,-1)  22 (-1,-1, 1)
 *   23 ( 1,-1, 1)  24 (-1, 1,-1)  25 (-1, 1, 1)  26 ( 1,-1,-1)
 * with weights 8/27, 2/27, 1/54, 1/216 (rest, axis, edge, corner).
 *
 * Cells: (x, y, z), x fastest; cell index c = (z * ny + y) * nx + x.
 *
 * State buffer layout (lbm_state_bytes): plane-blocked arrays of Q = 19 or 27
 * directions.  Each z-plane holds Q contiguous arrays of qstride elements
 * (qstride = nx*ny rounded up to 64, see lbm_qstride), and the planes follow
 * each other: element (q, x, y, z) at [(z * Q + q) * qstride + y * nx + x] of
 * the storage type, nz * Q * qstride elements in all.  What an element holds
 * depends on the dtype:
 *   LBM_F64, LBM_F32            f_q (post-collision)
 *   LBM_F32_SHIFTED             f_q - w_q
 *   LBM_F16_SHIFTED/BF16_SHIFTED  RNE(s (f_q - w_q)), s a per-context power
 *                               of two (lbm_scale), IEEE half / bfloat16
 * Two-grid contexts hold f*(x) at slot [q][x].  AA contexts alternate two
 * layouts; use lbm_get_pdfs for a canonical copy.  Adjoint fields use the
 * same layout with the adjoint dtype (LBM_F64 or LBM_F32).
 *
 * Solid cells (mask value nonzero) hold the rest state f_q = w_q, are never
 * updated, and report rho = u = 0.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameter                 */
    LBM_ENOMEM = -2,     /* small scratch allocation failed               */
    LBM_EHIP = -3,       /* a HIP runtime call failed                     */
    LBM_EDIVERGED = -4,  /* watchdog: NaN/Inf or mass drift beyond bound  */
    LBM_ESTATE = -5      /* call not valid for this context's set-up      */
} lbm_status;

/* Equilibria.  STANDARD: second-order part of eq. discreteEquilibriumStandard
 * (Sec. 2.2) with D3Q19 weights (D3Q19-S).  IMPROVED: eq.
 * new_d3q19_equilibrium (Sec. 3.2), built by matching 19 Maxwellian moments
 * (D3Q19-I).  Both use rho0 = 1 unless compressible is set (Sec. 2.3). */
enum { LBM_EQ_STANDARD = 0, LBM_EQ_IMPROVED = 1,
       /* IMPROVED3: the same construction carried to third order in u, i.e.
        * the equilibrium whose moments are the D3Q19-I column of Table 1
        * (Sec. 3.1) including its O(u^3) terms. */
       LBM_EQ_IMPROVED3 = 2 };

/* Collision.  SRT: eq. lb_srt_with_forces (Sec. 2.3).  TRT: two relaxation
 * rates, omega (even part) and omega_minus (odd part) with
 * Lambda = (1/omega - 1/2)(1/omega_minus - 1/2) = trt_magic; the force
 * term, which is odd, takes the factor (1 - omega_minus/2).  The paper names
 * TRT (Sec. 1, Sec. 3.3) without defining it.  MRT (D3Q19 only): the
 * collision C = -M^-1 S (M f - m_eq) + M^-1 (I - S/2) M F of Sec. 3.2 in the
 * space of the 19 monomial moments that D3Q19 keeps (all xi^e with
 * e_i in {0,1,2} except the 8 that Sec. 3.2 drops), with m_eq the moments of
 * the chosen equilibrium (for IMPROVED: the Maxwellian ones).  Rates:
 * second-order moments omega, third-order mrt_omega3, fourth-order
 * mrt_omega4 (conserved moments are unaffected by their rate).  KBC (D3Q19
 * only): the entropically stabilised collision that Sec. 3.3 adapts to the
 * Maxwellian moments and Sec. 5.2 uses at Re = 500 (Karlin, Boesch and
 * Chikatamarla 2014, the KBC-N4 split of Boesch et al. 2015), in the same 19
 * moments: the shear part (second- and third-order moments) relaxes at
 * omega, the fourth-order part at gamma omega / 2 with the stabiliser gamma
 * chosen per cell to minimise the entropy of the post-collision state to
 * second order about f^eq over 0 <= gamma <= 2 (gamma = 2 is SRT; the bound
 * keeps the fourth-order rate at or below omega).  The force enters as for
 * MRT. */
enum { LBM_SRT = 0, LBM_TRT = 1, LBM_MRT = 2, LBM_KBC = 3 };

/* Storage types of the PDF state. */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F32_SHIFTED = 2, LBM_F16_SHIFTED = 3,
       LBM_BF16_SHIFTED = 4 };

/* Rounding of the 16-bit stores s (f - w) (a6).  NEAREST: round to nearest
 * even.  STOCHASTIC: the FP32 value plus uniform random bits below the kept
 * mantissa, truncated toward zero, so the stored value is the lower or upper
 * neighbour with probabilities that make its expectation exact (FP16: below
 * 2^-14 s, its subnormal range, the last step is round to nearest).  The
 * random bits of f*_q(x) at step t are a counter-based hash of (seed, t, x,
 * q): runs are reproducible and both patterns store identical values.  With
 * round to nearest, a per-step change smaller than half a storage ulp of
 * s (f - w) is lost every step, which stalls a flow driven by a small body
 * force; stochastic rounding keeps it on average.  Ignored by the FP64 and
 * FP32 formats; the initial state and lbm_set_pdfs round to nearest. */
enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 };

/* Cache policy of the stream-collide and adjoint kernels.  STREAM:
 * non-temporal hints (each value is touched once per step; best when the
 * data is far larger than the 256 MB last-level cache).  KEEP: ordinary
 * cached accesses, so a lattice that fits the cache is served from it
 * between steps.  AUTO: KEEP for a kernel when one of its steps touches at
 * most 240 MiB (stream-collide: both buffers for two-grid, the one buffer
 * for AA; adjoint: the state and two adjoint fields), STREAM otherwise.
 * Results are identical bit for bit. */
enum { LBM_CACHE_AUTO = 0, LBM_CACHE_STREAM = 1, LBM_CACHE_KEEP = 2 };

/* What lbm_adjoint_step writes at solid cells.  COPY: lam_t = lam_{t+1}
 * there (solid cells keep their values through a step).  SKIP: nothing; for
 * callers that never read lambda at solid cells (fluid cells neither pull
 * from nor push into solid slots, lbm_objective writes zero there and
 * lbm_init_vjp returns zero there), it saves 2 Q sizeof(lambda) bytes per
 * solid cell and step. */
enum { LBM_ADJ_SOLID_COPY = 0, LBM_ADJ_SOLID_SKIP = 1 };

/* Streaming patterns.  TWO_GRID: pull from one buffer into another.  AA:
 * one buffer updated in place, alternating a step that reads and writes the
 * cell's own slots with a step that reads and writes the neighbours'. */
enum { LBM_TWO_GRID = 0, LBM_AA = 1 };

/* Objectives of lbm_objective. */
enum { LBM_OBJ_KINETIC_ENERGY = 0, LBM_OBJ_OUTLET_FLUX = 1 };

typedef struct {
    int32_t nx, ny, nz;       /* cells; nx*ny*nz < 2^31                           */
    int32_t periodic[3];      /* per axis: 1 periodic, 0 half-way bounce-back walls
                                 at both faces (Sec. 5.1)                        */
    int32_t equilibrium;      /* LBM_EQ_*                                         */
    int32_t collision;        /* LBM_SRT / LBM_TRT / LBM_MRT / LBM_KBC (D3Q19)    */
    int32_t dtype;            /* storage, LBM_F64 ... LBM_BF16_SHIFTED             */
    int32_t pattern;          /* LBM_TWO_GRID / LBM_AA                            */
    int32_t compressible;     /* 0: rho0 = 1 (the paper's choice); 1: rho0 = rho   */
    int32_t adjoint_dtype;    /* LBM_F64 (only with dtype LBM_F64) or LBM_F32      */
    int32_t stencil;          /* 19 (D3Q19) or 27 (D3Q27; its single equilibrium
                                 is the moment-matched = standard one, Sec. 3.1,
                                 whatever `equilibrium` says)                    */
    double omega;             /* SRT rate or TRT even rate, 0 < omega < 2         */
    double trt_magic;         /* TRT Lambda > 0; ignored for SRT                  */
    double accel[3];          /* body acceleration a; F_q = 3 w_q c_q.a (Sec. 2.3) */
    double scale;             /* F16/BF16: s (power of two) or 0 = chosen by
                                 lbm_init from the initial state                  */
    double mrt_omega3;        /* MRT rate of the third-order moments, (0, 2)      */
    double mrt_omega4;        /* MRT rate of the fourth-order moments, (0, 2)     */
    int32_t rounding;         /* LBM_ROUND_NEAREST / LBM_ROUND_STOCHASTIC          */
    uint32_t seed;            /* key of the stochastic rounding                    */
    int32_t cache_policy;     /* LBM_CACHE_AUTO / STREAM / KEEP                    */
    int32_t adjoint_solid;    /* LBM_ADJ_SOLID_COPY / SKIP                         */
    int32_t open_x;           /* 1: open x faces (Sec. 5.2): a velocity inlet at
                                 x = -1/2 (lbm_set_inlet) and a constant-pressure
                                 outlet at x = nx - 1/2; needs periodic[0] == 0,
                                 the two-grid pattern and compressible == 0      */
    double rho_out;           /* outlet density (open_x), > 0                      */
} lbm_params;

/* Library version string. */
const char *lbm_version(void);

/* Velocity set as encoded in the library for stencil 19 or 27:
 * c[Q*3], w[Q], opposite[Q]. */
void lbm_velocity_set(int32_t stencil, int32_t *c, double *w, int32_t *opposite);

/* qstride (elements between the direction arrays of one z-plane, see the
 * layout above) and bytes of one PDF state buffer and of one adjoint field,
 * for these parameters.  Host only; no GPU needed. */
int lbm_qstride(const lbm_params *p, int64_t *qstride);
int lbm_state_bytes(const lbm_params *p, size_t *bytes);
int lbm_adjoint_bytes(const lbm_params *p, size_t *bytes);

/* Validate p without touching the GPU.  LBM_OK or LBM_EINVAL; msg (may be
 * NULL) receives the reason, at most msg_len bytes. */
int lbm_validate(const lbm_params *p, char *msg, size_t msg_len);

/* Bytes of the link-word buffer that lbm_init needs for a lattice with a
 * solid mask: uint32 [cells] link words followed by uint32
 * [ceil(cells / 256)] for the list of 256-cell blocks that hold a fluid
 * cell.  Host only. */
int lbm_links_bytes(const lbm_params *p, size_t *bytes);

/* Storage scale s that lbm_init picks (scale == 0) for the 16-bit shifted
 * formats when the largest |f^eq_q - w_q| of the initial state is maxdev:
 * s = 2^floor(log2(1024 / maxdev)), clamped to [2^-10, 2^14]; 2^14 when
 * maxdev == 0.  FP16 keeps 11 significant bits whatever s is; s only keeps
 * s |f - w| inside the format's normal range, and 2^14 does so for every
 * |f - w| in [2^-28, 4), so a state near rest never gets a scale that the
 * developing flow would overflow.  Other dtypes: 1.  LBM_EINVAL when
 * maxdev is negative or not finite.  Host only. */
int lbm_choose_scale(int32_t dtype, double maxdev, double *scale);

/* Create a context and write the initial state.  The state of the method is
 * the set of populations f_q(x) of Sec. 2.3; the update of eq.
 * lb_srt_with_forces maps post-collision populations at t to those at
 * t + 1.  The initial state is f_q = f^eq_q(rho_init, u_init) of the chosen
 * equilibrium (eq. discreteEquilibriumStandard, Sec. 2.2, or eq.
 * new_d3q19_equilibrium, Sec. 3.2), with no force shift, stored as the
 * post-collision state at t = 0; solid cells hold f_q = w_q.
 *   solid    device uint8 [nz][ny][nx], nonzero = solid; NULL = all fluid.
 *            Read only during lbm_init; the caller may free or change it
 *            afterwards.
 *   links    device buffer of lbm_links_bytes bytes, caller-owned, required
 *            when solid is given (ignored otherwise): lbm_init writes one
 *            link word per cell into it (bit q: the pull source x - c_q is
 *            inside and fluid; bit 31: the cell is solid), which every
 *            kernel of the context reads, and after them the ascending list
 *            of the 256-cell blocks that hold a fluid cell: the
 *            stream-collide steps, and the adjoint with adjoint_solid ==
 *            SKIP, launch only those blocks.  Must outlive the context and
 *            stay unchanged.
 *   pdf0     device state buffer (lbm_state_bytes), caller-owned
 *   pdf1     second state buffer for TWO_GRID; must be NULL for AA
 *   stream   hipStream_t (NULL = default stream)
 *   rho_init device double [cells], or NULL for rho = 1
 *   u_init   device double [3][cells]
 * For F16/BF16 storage with scale == 0 the scale is lbm_choose_scale of the
 * largest |f^eq - w| over the initial state.  The library allocates only
 * small reduction scratch (about 32 bytes per 256 cells).  On failure *out
 * is NULL: LBM_EINVAL for invalid parameters or missing buffers, LBM_ENOMEM
 * when the scratch cannot be allocated, LBM_EHIP for a failed launch. */
int lbm_init(lbm_ctx **out, const lbm_params *p, const uint8_t *solid, uint32_t *links,
             void *pdf0, void *pdf1, void *stream, const double *rho_init, const double *u_init);

/* Release the context's scratch memory (not the caller's buffers). */
void lbm_destroy(lbm_ctx *c);

/* Message of the last failed call on this context (or of the last failed
 * lbm_init when c is NULL). */
const char *lbm_last_error(const lbm_ctx *c);

/* Advance nsteps >= 0 time steps: eq. lb_srt_with_forces with pull
 * streaming, half-way bounce-back at walls and solid cells, periodic wrap,
 * the chosen equilibrium and collision, the force F_q and the force-shifted
 * velocity of eq. macroscopic_vel_shift.  One fused kernel per step. */
int lbm_step(lbm_ctx *c, int64_t nsteps);

/* One two-grid step from src into dst (state buffers of this context's dtype
 * in the two-grid layout, src != dst), leaving the context's own state
 * untouched.  Used to recompute trajectories for the adjoint; allowed for
 * contexts of either pattern.  t >= 0 is the time of the state in src: the
 * step is the one lbm_step performs from time t, so with stochastic rounding
 * the result equals lbm_step's bit for bit.  LBM_EINVAL if src == dst or a
 * pointer is NULL or t < 0. */
int lbm_stream_collide(lbm_ctx *c, const void *src, void *dst, int64_t t);

/* Device pointer of the buffer that holds the current state. */
void *lbm_current_state(lbm_ctx *c);

/* Copy one state buffer (lbm_state_bytes bytes) from src to dst, e.g. to
 * take or restore a checkpoint.  Stream-ordered. */
int lbm_copy_state(lbm_ctx *c, const void *src, void *dst);

/* Steps taken since lbm_init (AA parity is its lowest bit). */
int64_t lbm_time(const lbm_ctx *c);

/* Storage scale s of F16/BF16 contexts (1 for the others). */
double lbm_scale(const lbm_ctx *c);

/* Macroscopic moments of the current state (Sec. 2.3): rho = sum_q f*_q and
 * u = (sum_q c_q f*_q - a/2) / rho0', which equals the equilibrium velocity
 * of the update that produced the state.  rho: device double [cells] or
 * NULL; u: device double [3][cells] or NULL; sums: host double[4] or NULL,
 * receives the FP64 totals over fluid cells of rho and of sum_q c_q f*_q
 * (mass and momentum); a non-NULL sums synchronises the stream. */
int lbm_moments(lbm_ctx *c, double *rho, double *u, double *sums);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * moments and FP64 totals of lbm_moments for a state buffer, without a
 * context, allocating nothing.  The reduction scratch is a fixed static
 * device array inside the library (16 MiB per GPU the library runs on, held
 * until the process ends), which limits the lattice to
 * LBM_NOALLOC_MAX_CELLS cells.  Every call on a GPU shares that array:
 * calls that overlap on one GPU (on different streams, or from different
 * threads) race and give wrong totals.  Results equal lbm_moments' bit for
 * bit (same kernels, same reduction order).
 *   p      the lattice's parameters
 *   links  the link words lbm_init wrote for a lattice with a solid mask;
 *          NULL for a lattice without one
 *   state  device state buffer in the layout the pattern holds after t
 *          steps (two-grid: direct; AA: t even local, t odd neighbour)
 *   t      steps taken since initialisation (the AA parity)
 *   scale  storage scale s of the 16-bit formats (lbm_scale); ignored for
 *          the others
 *   rho    device double [cells] or NULL; u device double [3][cells] or NULL
 *   sums   device double[4] or NULL: the FP64 totals over fluid cells of
 *          rho and of sum_q c_q f*_q, written (stream-ordered, no sync)
 *   stream hipStream_t (NULL = default stream)
 * LBM_EINVAL for invalid parameters, more than LBM_NOALLOC_MAX_CELLS cells,
 * a NULL state, t < 0 or a 16-bit scale that is not a power of two;
 * LBM_EHIP when the scratch's device address cannot be looked up or the
 * launch fails.  The message is lbm_last_error(NULL).  The array's device
 * address is looked up (hipGetSymbolAddress) once per GPU, by lbm_init or
 * else by this function's first call on that GPU: make that first call
 * outside a graph capture.  The successful path allocates nothing, on the
 * device or the host. */
#define LBM_NOALLOC_MAX_CELLS (1LL << 27)
int lbm_moments_noalloc(const lbm_params *p, const uint32_t *links, const void *state,
                        int64_t t, double scale, double *rho, double *u, double *sums,
                        void *stream);

/* Canonical copy of the current state: the post-collision populations f*_q
 * of Sec. 2.3 (the left side of eq. lb_srt_with_forces after the last step)
 * as device double [Q][cells] (dense, no padding, x fastest), in FP64
 * whatever the storage dtype and AA parity: dequantised as f = w + d / s
 * for the shifted formats; solid cells give w_q.  LBM_EINVAL for a NULL
 * pointer; stream-ordered. */
int lbm_get_pdfs(lbm_ctx *c, double *canonical);

/* Canonical f*_q (FP64) of the current state at n listed cells: cells is a
 * device int64 [n] of cell indices, out a device double [n][Q].  Indices
 * outside the lattice give NaN rows.  For probing states too large to copy
 * whole. */
int lbm_sample_pdfs(lbm_ctx *c, const int64_t *cells, int64_t n, double *out);

/* Overwrite the current state (the populations f*_q of Sec. 2.3, as
 * lbm_get_pdfs returns them) from a canonical device double [Q][cells]:
 * stored as f (FP64, FP32) or quantised as RNE(s (f - w)) (shifted formats,
 * the context's scale), in the layout the context's pattern and step parity
 * need.  Solid cells are set to w_q.  LBM_EINVAL for a NULL pointer;
 * stream-ordered. */
int lbm_set_pdfs(lbm_ctx *c, const double *canonical);

/* Watchdog: FP64 mass of the current state against the mass at lbm_init.
 * LBM_EDIVERGED if a total is not finite or |mass - mass0| > rel_tol mass0.
 * Synchronises the stream. */
int lbm_watchdog(lbm_ctx *c, double rel_tol);

/* Change omega and the body acceleration of an existing context. */
int lbm_set_rates(lbm_ctx *c, double omega, const double *accel);

/* Inflow velocity of a context with open x faces (Sec. 5.2, where a parabolic
 * profile is prescribed at the inflow): u_in is a device double [3][nz][ny],
 * component-major, the velocity of the inlet cell (0, y, z); caller-owned,
 * borrowed until the next lbm_set_inlet or lbm_destroy, read by every step.
 * A pull of cell (0, y, z) from beyond the inlet face takes Ladd's
 * moving-wall half-way bounce-back, g_q = f*_qbar + 6 w_q c_q . u_in(y, z)
 * (rho0 = 1); a pull of cell (nx-1, y, z) from beyond the outlet face takes
 * the anti-bounce-back of Ginzburg, Verhaeghe and d'Humieres,
 * g_q = -f*_qbar + 2 f^eq+_q(rho_out, u_b), with f^eq+ the even part of the
 * equilibrium and u_b the read-out velocity of the cell's stored state.
 * lbm_step and lbm_stream_collide return LBM_ESTATE for an open context
 * until this has been called; LBM_ESTATE for a context without open faces,
 * LBM_EINVAL for NULL. */
int lbm_set_inlet(lbm_ctx *c, const double *u_in);

/* ------------------------------------------------------------------------ */
/* Adjoint (not in the paper): exact transpose of one two-grid step, for    */
/* every stencil and equilibrium and the SRT, TRT and MRT collisions of the */
/* forward step.  Adjoint fields hold Q arrays like a state.                */
/* Incompressible form (compressible == 0) without KBC or open faces only;  */
/* otherwise LBM_ESTATE.                                                    */
/* ------------------------------------------------------------------------ */

/* lam_prev = (d step / d f_t)^T lam_next for the step f_t -> f_{t+1}.
 *   state_t   device state buffer (context dtype, two-grid layout) holding
 *             f_t; the adjoint linearises at its dequantised values
 *   lam_next  device adjoint field (adjoint dtype) at t + 1
 *   lam_prev  device adjoint field at t (written; distinct from lam_next)
 *   grad      device double[4] or NULL: += dJ/domega, dJ/da_x, dJ/da_y,
 *             dJ/da_z of this step (FP64, deterministic order).  For TRT,
 *             omega_minus follows omega at fixed Lambda; for MRT omega is
 *             the rate of the second-order moments (mrt_omega3/4 fixed).
 * Per cell: gather as the forward step, mu = J_C^T lam_next, then write mu_r
 * to lam_prev[r] at x - c_r, or to lam_prev[opposite(r)] at x when x - c_r
 * is a wall or solid (every slot is written exactly once; no atomics).
 * Solid cells copy lam_next through, or are left unwritten (adjoint_solid).
 * LBM_ESTATE when state_t is the buffer of an AA context (it holds an AA
 * layout, not the two-grid one; lbm_stream_collide writes two-grid states
 * for either pattern). */
int lbm_adjoint_step(lbm_ctx *c, const void *state_t, const void *lam_next, void *lam_prev,
                     double *grad);

/* Objective J of a stored state and its seed lam_T = dJ/df_T.
 *   kind  LBM_OBJ_KINETIC_ENERGY: J = 1/2 sum over fluid cells of |u|^2
 *         LBM_OBJ_OUTLET_FLUX:    J = sum of u_x over fluid cells of x = nx-1
 *         with u the stored-state velocity of lbm_moments (rho0 = 1).
 *   state device state buffer of this context in the two-grid layout
 *         (LBM_ESTATE for the buffer of an AA context, which holds an AA
 *         layout)
 *   out   device double[4]: J and its explicit derivative dJ/da (through
 *         u = sum c f - a/2); written (not accumulated)
 *   lam   device adjoint field (written)                                      */
int lbm_objective(lbm_ctx *c, int kind, const void *state, double *out, void *lam);

/* Gradient with respect to u_init of f_0 = f^eq(1, u_init):
 * grad_u[b][x] = sum_q lam0_q(x) d f^eq_q / d u_b (device double [3][cells],
 * written; zero in solid cells).  u_init: device double [3][cells]. */
int lbm_init_vjp(lbm_ctx *c, const double *u_init, const void *lam0, double *grad_u);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
