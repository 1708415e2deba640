/*
 * lbm.h - C ABI of liblbm.so: one MI355X (gfx950) time step of the
 * thread-safe, high-order lattice Boltzmann solver coupled to a conservative
 * Allen-Cahn phase field, for droplet and bubble flows at high density and
 * viscosity contrast (Lauricella et al., arXiv 2501.00846).
 *
 * Physics (paper sections):
 *   Sec. II.A  incompressible two-phase Navier-Stokes with the potential-form
 *              surface force F^s = mu_phi grad(phi) (Eq. jaqminforce), and the
 *              conservative Allen-Cahn equation for phi in [0, 1], stepped by
 *              FTCS on the same grid.
 *   Sec. II.B  D3Q27 lattice, third-order Hermite equilibrium (Eq. eqts),
 *              recursively regularised non-equilibrium (Eq. noneqts), Guo
 *              source (Eq. guoforce); fused stream-and-collide from moments
 *              only (Eq. pushLB), so no population array is stored.
 *   Sec. II.C  force split F = F^s + F^p + F^nu (Eqs. press_corr,
 *              visc_corr), rho = rho_l phi + (1 - phi) rho_g, isotropic FD
 *              gradient and Laplacian.
 *   Sec. II.D  the four phases of one step.
 *   Sec. III   body force on the light phase, no-slip walls with a
 *              neutral-wetting (Robin) phase-field condition.
 *
 * Conventions for every host array passed through this ABI:
 *   - C order with x fastest: node index n = x + nx*(y + ny*z);
 *   - vectors are three SoA planes (x plane, then y, then z), 3*N doubles;
 *   - host arrays are owned by the caller and only read/written during the call.
 * Lattice units throughout: dx = dt = 1, c_s^2 = 1/3.
 *
 * State per node (11 scalars, the thread-safe moment set):
 *   phi, P = p* (= sum f), J = sum f c (3), Q = sum f (c c - c_s^2 I) - J J (6,
 *   ordered xx, yy, zz, xy, xz, yz).  Velocity is u = J + a/2, a = F/rho.
 *
 * Errors: every entry point returns lbm_status (0 = success, negative =
 * failure); no exception crosses the ABI.  Argument checks run on the host
 * before any device work, so they can be exercised without a GPU.  The text of
 * the last error of a context is returned by lbm_last_error (errors raised
 * before a context exists are reported by lbm_last_error(NULL)).
 * A context is used by one host thread at a time; calls on one context are not
 * thread-safe.  All device work of a context is ordered on its stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque; owned by the library */

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,         /* invalid argument (NULL, sizes, parameter ranges) */
  LBM_ERR_UNSUPPORTED = -2, /* valid but not provided (lattice, mixed precisions) */
  LBM_ERR_OOM = -3,         /* device allocation failed */
  LBM_ERR_DEVICE = -4,      /* a HIP call failed */
  LBM_ERR_UNSTABLE = -5,    /* non-finite state detected (NaN / Inf) */
  LBM_ERR_STATE = -6        /* call out of order (e.g. step before init) */
} lbm_status;

typedef enum { LBM_D3Q27 = 0 } lbm_lattice; /* D3Q27 (Sec. I, II.B); others -> UNSUPPORTED */

typedef enum {
  LBM_PERIODIC = 0,
  LBM_WALL = 1 /* no-slip half-way bounce-back + zero normal derivative of phi */
} lbm_bc;

typedef enum {
  LBM_FP64 = 0,    /* FP64 storage and arithmetic */
  LBM_FP32 = 1,    /* FP32 storage and arithmetic */
  LBM_FP16_OS = 2, /* phi FP32; 10 moments FP16 offset-and-scale; FP32 arithmetic */
  LBM_BF16_OS = 3  /* phi FP32; 10 moments BF16 offset-and-scale; FP32 arithmetic */
} lbm_precision;

enum {
  /* Advect phi with u.grad(phi) as printed in the FTCS update of Sec. II.D
   * instead of the conservative flux form div(phi u). */
  LBM_LITERAL_ADVECTION = 1,
  /* Gradient closure: rebuild the non-equilibrium second moment from the
   * velocity gradient, a2 = -(cs^2/omega)(grad J + grad J^T) (the
   * velocity-gradient a2 given with Eq. noneqts; J = sum f c, isotropic
   * gradient of Sec. II.C), also in the viscous correction (Eq. visc_corr).
   * The state is then phi, P, J only: 5 stored fields per node instead of
   * 11, and the Q fields of lbm_get_state read 0 (lbm_set_state ignores
   * them).  All boxes of a context must agree on this flag. */
  LBM_GRADIENT_CLOSURE = 2,
  /* Fourth-order phase-field update: the divergence, Laplacian and normal
   * gradient of the Allen-Cahn FTCS update become (4 D1 - D2)/3, the
   * isotropic D3Q27 stencil at spacings 1 and 2 (the higher-order
   * discretisation named as future work at the end of Sec. II.A; the flow
   * solver keeps the second-order stencils of Sec. II.C).  Wall axes need
   * at least 4 nodes.  Each step then also keeps 6 values per node of
   * device memory in the phi storage type (velocity and sharpening flux of
   * level n), runs two more kernels, and computes the phase update in the
   * precision of the stored phi.  All boxes of a context must agree on this flag and, with
   * it, on LBM_LITERAL_ADVECTION; not available through lbm_step_noalloc. */
  LBM_HIGH_ORDER_AC = 4,
  /* Finer phase-field grid (the finer grid named as future work at the end
   * of Sec. II.A): phi lives on a grid refined by 2 per axis, cell centred
   * (fine nodes 2i and 2i + 1 at i - 1/4 and i + 1/4 of coarse node i,
   * spacing 1/2), and is advanced by the FTCS update of Sec. II.D with the
   * stencils of Sec. II.C at that spacing and the trilinear interpolation of
   * the coarse velocity; the flow solver reads the coarse phi, the mean of
   * the 8 fine nodes of each cell.  A phi given to lbm_init_phase or
   * lbm_set_state is carried to the fine grid by the same interpolation and
   * the coarse phi becomes its restriction; lbm_get_fine_phase /
   * lbm_set_fine_phase read and write the fine field itself.  The diffusive
   * part of the fine FTCS update is stable for mobility <= 0.0865 (larger
   * values are rejected with LBM_ERR_ARG).  Each box keeps two
   * fine phi buffers (8 N values of the phi storage type each) and the coarse
   * velocity (3 N values of that type); a step runs three more kernels.  All
   * boxes of a context must agree on this flag; not combined with LBM_HIGH_ORDER_AC or
   * LBM_LITERAL_ADVECTION, and not available through lbm_step_noalloc. */
  LBM_FINE_PHASE = 8
};

/* One box.  phi = 1 is the liquid (subscript l), phi = 0 the gas (g). */
typedef struct {
  int32_t nx, ny, nz;     /* 1 .. 2^20; >= 2 on an axis with walls; nx rounded
                             up to a multiple of 32, times ny, <= 2^28 */
  int32_t lattice;        /* lbm_lattice */
  int32_t bc[3];          /* lbm_bc per axis x, y, z */
  int32_t precision;      /* lbm_precision; identical for all boxes of a context */
  int32_t flags;          /* LBM_LITERAL_ADVECTION | LBM_GRADIENT_CLOSURE | LBM_HIGH_ORDER_AC |
                             LBM_FINE_PHASE, or 0 */
  double rho_l, rho_g;    /* phase densities, > 0 (Sec. II.C) */
  double nu_l, nu_g;      /* kinematic viscosities, > 0; omega = 1/(3 nu + 1/2) */
  double sigma;           /* surface tension, >= 0 (Sec. II.C: beta = 12 sigma/W, kappa = 3 sigma W/2) */
  double mobility;        /* Allen-Cahn diffusivity D = M, >= 0, FTCS-stable if <= 0.34 */
  double width;           /* interface width W (the paper's delta), > 0 */
  double gravity[3];      /* body force density (rho - rho_ref) * gravity (Sec. III.A) */
  double rho_ref;
} lbm_params;

/* Device resources.  stream: a hipStream_t on which every kernel and copy of
 * the context is enqueued (NULL: the library creates a stream of its own).
 * alloc/free: device allocator callbacks (NULL: hipMalloc / hipFree); alloc
 * returns device memory of at least `bytes` bytes aligned to 256 bytes, or
 * NULL on failure.  user is passed back unchanged. */
typedef struct {
  void* stream;
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} lbm_device;

/* Reductions over one box, accumulated in FP64 on the device. */
typedef struct {
  double phase_mass;      /* sum phi */
  double pstar_sum;       /* sum p* */
  double momentum[3];     /* sum rho u */
  double kinetic;         /* 1/2 sum rho |u|^2 */
  double umax;            /* max |u| */
  double centroid_l[3];   /* sum phi x / sum phi */
  double velocity_l[3];   /* sum phi u / sum phi */
  double centroid_g[3];   /* sum (1-phi) x / sum (1-phi) */
  double velocity_g[3];   /* sum (1-phi) u / sum (1-phi) (bubble centre-of-mass velocity) */
  double p_l, p_g;        /* mean p = rho c_s^2 p* over bulk nodes phi >= 0.98 / phi <= 0.02 */
  double n_l, n_g;        /* number of those bulk nodes */
  int32_t nonfinite;      /* 1 if any state value is NaN or Inf */
} lbm_diag;

/* Tile / launch configuration of the fused step (chosen by lbm_autotune). */
typedef struct {
  int32_t block_x, block_y; /* workgroup columns; supported pairs: (32,8) (34,8) (34,15); with the moment closure also (18,14), and (66,8) except in FP64 */
  int32_t z_chunk;          /* planes marched by one workgroup, >= 1 */
  int32_t persistent;       /* 0: one workgroup per tile; n > 0: n workgroups loop over tiles */
} lbm_tuning;

/* Create a context holding n_boxes >= 1 independent boxes stepped together
 * (one launch per step covers every box).  Each lbm_params is the paper's
 * statement of one problem: the grid and the D3Q27 lattice (Sec. II.B, Eq.
 * lbe), the two phases' densities and viscosities (Sec. II.A, Eq. NSeq; the
 * density law below Eq. press_corr), the surface tension through beta and
 * kappa of the chemical potential (Sec. II.C), the Allen-Cahn diffusivity D
 * and interface width delta (Sec. II.A), the body force on the light phase
 * and the no-slip walls (Sec. III.A, III.D).  All parameters are validated
 * before any device call.  The state is undefined until lbm_init_phase or
 * lbm_set_state has been called for every box.  On success *out owns all
 * device memory of the state (2 x 11 fields per box, ping-pong; 2 x 5 with
 * LBM_GRADIENT_CLOSURE).  On the device each stored row of nx nodes is padded
 * to a 64-byte multiple (at most 31 unused elements per row), so that every
 * row of every field starts on a 64-byte boundary. */
lbm_status lbm_create(const lbm_params* boxes, int32_t n_boxes, const lbm_device* dev,
                      lbm_ctx** out);

/* Initial state of one box (Sec. II.D; P = p*_0, J = u_0, Q = 0).
 * phi: N doubles (required); u: 3N doubles or NULL (0); pstar: N doubles or
 * NULL (0).  N = nx*ny*nz of that box.  Blocks until the copy is done. */
lbm_status lbm_init_phase(lbm_ctx* ctx, int32_t box, const double* phi, const double* u,
                          const double* pstar);

/* Enqueue nsteps >= 0 time steps of every box on the context stream
 * (replayed from a captured hipGraph when graphs are enabled). Asynchronous.
 * One step is the four phases of Sec. II.D: moments and forces (Eqs.
 * moments0, moments1, press_corr, jaqminforce, visc_corr), pre-regularisation
 * (Eq. hermite_neq2), the fused stream-collide (Eqs. LBexp, pushLB, eqts,
 * noneqts, guoforce), taken as a pull so that each thread writes only its
 * own node (the thread-safe principle of Sec. II.B), and the FTCS update of
 * the conservative Allen-Cahn equation (Sec. II.A, update formula of
 * Sec. II.D).  Errors: LBM_ERR_STATE if a box has no state yet;
 * LBM_ERR_DEVICE if a launch fails.  A step that goes non-finite is reported
 * by the next lbm_get_fields / lbm_diagnostics. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Observables of one box (Sec. II.C): rho = rho_l phi + (1-phi) rho_g,
 * u = J + a/2 (3N, SoA), phi, p = rho c_s^2 p*.  Any pointer may be NULL.
 * Synchronises the stream.  Returns LBM_ERR_UNSTABLE (with outputs written)
 * if the state holds a non-finite value. */
lbm_status lbm_get_fields(lbm_ctx* ctx, int32_t box, double* rho, double* u, double* phi,
                          double* p);

/* FP64 reductions of one box: phase mass and sum p* (conserved by the flux
 * form of Sec. II.A and the moments of Eq. moments0), momentum and kinetic
 * energy with u = J + a/2 (Eq. moments1), the centroid and centre-of-mass
 * velocity of each phase (the bubble rise velocity compared in Sec. III.A,
 * Fig. comparison), and the bulk pressures p = rho cs^2 p* (Sec. II.C, below
 * Eq. press_corr) from which the Laplace jump is read.  *out is written
 * whenever the reduction ran.  Synchronises; LBM_ERR_UNSTABLE if nonfinite. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, int32_t box, lbm_diag* out);

/* The reductions of lbm_diagnostics for every box of the context from one
 * launch (an ensemble's observables at the cost of one call): out holds
 * n_boxes structs, box after box, each bitwise equal to what
 * lbm_diagnostics returns for that box.  Synchronises; LBM_ERR_UNSTABLE
 * (every struct written) if any box holds a non-finite value. */
lbm_status lbm_diagnostics_all(lbm_ctx* ctx, lbm_diag* out);

/* Raw state of one box as 11 N-double planes in the order
 * phi, P, Jx, Jy, Jz, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz (decoded to FP64).
 * get synchronises; set replaces the state (checkpoint / restart). */
lbm_status lbm_get_state(lbm_ctx* ctx, int32_t box, double* state);
lbm_status lbm_set_state(lbm_ctx* ctx, int32_t box, const double* state);

/* Raw state (decoded to FP64) at n chosen nodes of one box: node[j] is a
 * flat index x + nx*(y + ny*z) in [0, N); out holds 11 planes of n doubles in
 * the field order of lbm_get_state (out[k*n + j]).  For spot checks of large
 * boxes without copying the whole state.  Synchronises. */
lbm_status lbm_get_state_points(lbm_ctx* ctx, int32_t box, int64_t n, const int64_t* node,
                                double* out);

/* The fine phase field of a box created with LBM_FINE_PHASE: 8 N doubles,
 * index X + 2nx (Y + 2ny Z) over the fine grid (2nx x 2ny x 2nz, node X at
 * X/2 - 1/4 in lattice units).  get synchronises and reports
 * LBM_ERR_UNSTABLE for non-finite values; set replaces the fine field of a
 * box that holds a state (LBM_ERR_STATE otherwise) and sets the coarse phi
 * to its restriction (an exact restart together with lbm_set_state of the
 * other fields first).  LBM_ERR_UNSUPPORTED for a box without the flag. */
lbm_status lbm_get_fine_phase(lbm_ctx* ctx, int32_t box, double* out);
lbm_status lbm_set_fine_phase(lbm_ctx* ctx, int32_t box, const double* in);

/* The fine phase field (decoded to FP64) at n chosen fine nodes of a box
 * created with LBM_FINE_PHASE: node[j] is a flat fine index
 * X + 2nx (Y + 2ny Z) in [0, 8 N), out[j] its value.  For spot checks of
 * large boxes without copying the whole fine field.  Synchronises.
 * LBM_ERR_ARG for an index out of range, LBM_ERR_STATE before the box holds
 * a state, LBM_ERR_UNSUPPORTED for a box without the flag. */
lbm_status lbm_get_fine_phase_points(lbm_ctx* ctx, int32_t box, int64_t n, const int64_t* node,
                                     double* out);

/* Offset-and-scale encoding of the 10 moments of one box in the 16-bit
 * storage modes: stored = (value - offset[k]) * scale[k], k over P, Jx, Jy, Jz,
 * Qxx, Qyy, Qzz, Qxy, Qxz, Qyz, computed in FP32 and rounded to nearest even.
 * scale must be a power of two in [2^-126, 2^126] and offset finite in FP32.
 * Without a call, offsets are 0 and scales 1024 (P), 4096
 * (J), 65536 (Q).  If the box already holds a state, that state is re-encoded
 * on the device (decoded with the previous offsets and scales, encoded with
 * the new ones), so its values change only by the rounding of the new
 * encoding; the next step uses the new encoding.  If the re-encoding fails on
 * the device (LBM_ERR_DEVICE), the box has no valid state until the next
 * lbm_init_phase / lbm_set_state.  Synchronises.  Ignored in
 * the FP64 and FP32 modes (returns LBM_OK).  The storage precision is the
 * paper's silence: Sec. II.B fixes the moment set, not its format. */
lbm_status lbm_set_encoding(lbm_ctx* ctx, int32_t box, const double* offset,
                            const double* scale);

/* Launch configuration of the fused step. */
lbm_status lbm_set_tuning(lbm_ctx* ctx, const lbm_tuning* t);
lbm_status lbm_get_tuning(const lbm_ctx* ctx, lbm_tuning* t);

/* Time each supported tuning for `steps` steps (each after two warm-up
 * steps), time the finalists within 5 % of the fastest twice more (over
 * 2*steps steps, or enough steps to span ~25 ms, at most 4096), and keep the
 * tuning with the best time per step.  Advances
 * the state by every step it runs.  Writes the choice to *best if non-NULL.
 * On an error the previous tuning stays in place. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t steps, lbm_tuning* best);

/* Enable (1, default) or disable (0) hipGraph capture of lbm_step. */
lbm_status lbm_set_graphs(lbm_ctx* ctx, int32_t enabled);

/* Enqueue one separate launch of the fused step per box per step instead of
 * one launch covering all boxes (the unbatched baseline of an ensemble). */
lbm_status lbm_step_unbatched(lbm_ctx* ctx, int32_t nsteps);

/* Wait for all work enqueued on the context stream. */
lbm_status lbm_synchronize(lbm_ctx* ctx);

/* Algorithmic HBM bytes per lattice update of the fused step in this
 * context's precision (11 fields read + 11 written). */
double lbm_bytes_per_update(const lbm_ctx* ctx);

/* Total nodes over all boxes. */
int64_t lbm_total_nodes(const lbm_ctx* ctx);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): enqueue
 * nsteps >= 0 fused steps of ONE box whose state lives in device buffers the
 * caller owns, with no context and no allocation of any kind.  The step is
 * the one lbm_step runs (same kernels, bitwise the same results); only the
 * descriptor and the tile list it reads live in a fixed array of the library
 * (1 MiB of device memory per GPU, held until the process ends; at most
 * 32,736 tiles, else LBM_ERR_ARG: use a larger z_chunk).
 *
 * box: parameters, checked as by lbm_create (the precision is the storage).
 * tuning: launch configuration as in lbm_set_tuning, or NULL (34 x 15 tiles,
 *   a z-chunk that fills the GPU and fits the tile limit).
 * phi[s], mom[s], s = 0, 1: the two ping-pong state buffers, each aligned to
 *   its element size (64-byte alignment enables the non-temporal stores):
 *   pitch = nx rounded up to a multiple of 8 (FP64), 16 (FP32) or 32 (16-bit
 *   modes) elements;
 *   phi[s]: nz*ny*pitch elements, FP64 in LBM_FP64 else FP32; node (x, y, z)
 *     at (z*ny + y)*pitch + x;
 *   mom[s]: nz*nmom*ny*pitch elements, FP64 / FP32 / IEEE binary16 / bfloat16
 *     by precision, k over P, Jx, Jy, Jz, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz
 *     (nmom = 10), or P, J (nmom = 4) with LBM_GRADIENT_CLOSURE.  FP64 and
 *     FP32: moment k of node (x, y, z) at ((z*nmom + k)*ny + y)*pitch + x.
 *     16-bit modes: moments in pairs (k = 2p, 2p + 1), one 32-bit word per
 *     node and pair with the even field in the low half, moment k at 16-bit
 *     element 2*(((z*nmom/2 + k/2)*ny + y)*pitch + x) + k%2; each stores
 *     (value - enc_offset[k]) * enc_scale[k].
 *   Elements x >= nx of a row are never read or written.
 * enc_offset, enc_scale: 10 values each (rules of lbm_set_encoding) or both
 *   NULL (the default encoding); ignored outside the 16-bit modes.
 * parity: the buffer holding the current state; after the call the state is
 *   in buffer parity ^ (nsteps & 1), and every node of it is written.
 * stream: the hipStream_t the work is enqueued on (NULL: the null stream).
 *   Asynchronous; no synchronisation.
 * All argument checks run before any device call; errors are reported by
 * lbm_last_error(NULL).  Every call on one GPU shares that GPU's descriptor
 * and tile list, rewritten by each call: calls whose work overlaps on one GPU
 * (different streams, or host threads) race and must be serialised. */
lbm_status lbm_step_noalloc(const lbm_params* box, const lbm_tuning* tuning, void* const phi[2],
                            void* const mom[2], const double* enc_offset, const double* enc_scale,
                            int32_t parity, int32_t nsteps, void* stream);

/* Release every device resource of the context.  NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* Text of the last error on ctx (or of the last failed lbm_create when ctx is
 * NULL).  Valid until the next call on the same context. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
