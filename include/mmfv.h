/*
 * mmfv.h -- C ABI of the MI355X (gfx950) library for the conservative
 * sharp-interface method for compressible multi-material flows of Pan, Han,
 * Hu & Adams (arXiv:1704.00519).
 *
 * One context advances one uniform-grid problem (1D or 2D) of up to
 * MM_MAX_MAT materials, each with its own stiffened-gas EOS, in FP64 on one
 * GPU.  The state is the regional level set (unsigned distance phi >= 0 and
 * integer indicator chi, Sec. 2.2) plus, per material r, the conserved cell
 * averages Q^r = alpha^r U^r (Eq. discretized_equ).  One call of mm_step
 * advances whole time steps of the method: cut-cell geometry from the level
 * set (Sec. 2.3), volume-fraction correction in cells of three or more
 * materials (Sec. 2.3.1, Eq. vol_corr2), per-material WENO5 / HLLC fluxes
 * scaled by apertures, the reduced interface-exchange model (Sec. 2.3.2),
 * the multi-region level-set advance (Sec. 2.2, Eq. local-advection and
 * Eq. reconstruction), mixing of small/new/vanishing cells after every
 * Runge-Kutta sub-step, with the third-order SSP Runge-Kutta scheme in the
 * beta-form of Eq. local-advection.
 *
 * Conventions
 *   Arrays crossing the ABI are C-ordered, interior cells only:
 *     phi, chi   [ny][nx]
 *     W, Q       [n_mat][dim+2][ny][nx], components (rho, u, [v], p) for W and
 *                (rho, rho u, [rho v], rho E) for Q = alpha U
 *     alpha      [n_mat][ny][nx]
 *   ny = 1 in 1D.  ptr_kind says whether pointers are host (MM_HOST) or
 *   device (MM_DEVICE) memory of the context's GPU; device pointers may be
 *   torch tensors' data_ptr().  Pointers are borrowed for the call only.
 *   All work is enqueued on the stream given to mm_create; calls that return
 *   data to host memory, or report errors, synchronise that stream.
 *
 * Errors: every function returns an mm_status; no exceptions cross the ABI.
 * mm_last_error() gives a message for the last failure on a context.
 */
#ifndef MMFV_H
#define MMFV_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_EINVAL = 1,    /* bad argument or configuration; nothing was changed  */
  MM_ENOMEM = 2,    /* device allocation failed                            */
  MM_EDEVICE = 3,   /* HIP runtime error                                   */
  MM_ENONPHYS = 4,  /* rho <= 0, p + p_inf <= 0 or non-finite in a real cell */
  MM_ESTATE = 5,    /* call order (e.g. mm_step before mm_init_state)      */
  MM_ENOTIMPL = 6   /* entry point declared but not available              */
} mm_status;

enum { MM_BC_TRANSMISSIVE = 0, MM_BC_REFLECTIVE = 1, MM_BC_INFLOW = 2,
       MM_BC_OUTFLOW = 3 };
enum { MM_HOST = 0, MM_DEVICE = 1 };
#define MM_MAX_MAT 8

/* Problem description (plain old data, caller-owned, copied by mm_create). */
typedef struct {
  int32_t dim, nx, ny, n_mat;    /* dim 1 or 2; ny = 1 when dim = 1         */
  double x0, x1, y0, y1;         /* domain; cells are (x1-x0)/nx wide       */
  double gamma[MM_MAX_MAT];      /* stiffened gas: p = (gamma-1) rho e      */
  double pinf[MM_MAX_MAT];       /*                    - gamma p_inf        */
  int32_t bc[4];                 /* MM_BC_* of x-lo, x-hi, y-lo, y-hi       */
  double inflow_W[4];            /* (rho, u, v, p) on MM_BC_INFLOW sides    */
  int32_t inflow_mat, rk_order;  /* material of the inflow; 3 (or 2)        */
  double cfl, alpha_mix;         /* CFL number (0.6); mixing threshold 0.5  */
  int32_t k_ext, band_ls;        /* upwind ghost sweeps (8); band width in  */
                                 /* cells of the level set (8)              */
  /* Tait materials (Sec. 2.1, Tait's equation for water-like fluids):
   * eos[m] = MM_EOS_TAIT gives p = B (rho/rho0)^gamma - B + p0 (pressure
   * from density alone; gamma[m] is the Tait exponent, pinf[m] unused) with
   * the energy relation of the stiffened gas of the same gamma and
   * p_inf = B - p0.  All zero: every material a stiffened gas. */
  int32_t eos[MM_MAX_MAT];
  double rho0[MM_MAX_MAT], tait_B[MM_MAX_MAT], p0[MM_MAX_MAT];
  int32_t flux;                  /* MM_FLUX_HLLC (0): component-wise WENO5 + */
                                 /* HLLC; MM_FLUX_ROE (1): characteristic-  */
                                 /* wise WENO5 + Roe                        */
  /* 1: the interface scale-separation model (Sec. 2.3.3) after every time
   * step.  Oddball cells, cut cells whose material has no cell crossed by
   * its contour shifted 0.75 h inwards within their 3 x 3 block, go to the
   * other material of largest volume fraction when that one is resolved in
   * the block; their distance is re-assigned from the outward-shifted
   * contour of the new material and their conserved quantities join it. */
  int32_t scale_sep;
  /* 1D cylindrical geometry and free surfaces (Sec. 3, Case II: the
   * implosion driven by a pressure on the shell's outer surface).
   * coord = 1 (dim 1, x0 >= 0): x is the radius; faces have the area
   * r_{i+-1/2}, cells the volume r_i dx, the radial momentum takes the
   * geometric source alpha p / r_i, a cut cell's interface area follows
   * from its faces and volume fraction, mixing exchanges r-weighted content,
   * and the diagnostics' sum_Q, bnd_in and exch are totals of r_i Q_i.
   * fs_on = 1 (dim 1, stiffened gases, HLLC): material fs_mat is an ambient
   * that is not solved.  At every stage its state is density fs_p[4] at
   * rest under p(t) (p(t) = fs_p[0] up to t = fs_p[2], linear to fs_p[1] at
   * t = fs_p[3] > fs_p[2], fs_p[1] afterwards); its conserved quantities are
   * alpha times that state; it has no fluxes and exchanges nothing; its
   * interfaces are free surfaces whose pressure is p(t) and whose velocity
   * is the solved side's wave jump to p(t); the step size also counts that
   * wave.  All zero: planar geometry, every material solved.  The adjoint
   * (record_tape) is not built for either. */
  int32_t coord, fs_on, fs_mat;
  double fs_p[5];
  /* 1 (dim 2, band_ls <= 10): redistancing of the level set after every
   * time step (after the scale separation).  Band cells (phi below the band
   * width) take new distances, the others keep the band width, the
   * material indicator stays: a cell with a 4-neighbour of another material
   * takes, per axis, the distance to the crossing of the local level set
   * between the two centres, h phi_c / (phi_c + phi_n) (h/2 where both are
   * 0), the smaller side; with crossings on both axes the distance to the
   * line through them, d_x d_y / sqrt(d_x^2 + d_y^2) (0 if one is 0), else
   * the one crossing; band_ls + 1 Jacobi sweeps then take the smallest of a
   * band cell's value and its same-material 8-neighbours' values plus the
   * centre distance, capped at the band width; geometry and correction are
   * evaluated again.  The paper describes no reinitialisation; without it
   * the distance degenerates in stretched layers.  The adjoint (record_tape)
   * is not built for it. */
  int32_t reinit;
} mm_config;
enum { MM_EOS_STIFFENED = 0, MM_EOS_TAIT = 1 };
enum { MM_FLUX_HLLC = 0, MM_FLUX_ROE = 1 };

/* Diagnostics of a context (mm_get_diagnostics). */
typedef struct {
  double t, dt;            /* time reached, last step size                  */
  int64_t steps;           /* time steps taken                              */
  int64_t n_posfix;        /* faces that fell back to first-order states    */
  int64_t n_fluxskip;      /* faces with A > 0 whose cells had no state     */
  int64_t n_ifskip;        /* interfaces skipped for lack of a ghost state  */
  int64_t n_stranded;      /* mixing sources without an eligible target     */
                           /* left in place (no other material to join)    */
  int64_t n_mixsrc;        /* mixing sources processed                      */
  int64_t n_updates;       /* active material-cell RK-substep updates       */
  int64_t err_cell;        /* j*nx+i of the lowest non-physical real cell   */
                           /* found, -1 if none                             */
  /* Conservation book-keeping (Eq. discretized_equ, Sec. 2.3.2: a material's
   * total changes only through the domain boundary and its exchange term),
   * per material and component (rho, rho u, rho v, rho E; rho v = 0 in 1D):
   * sum_Q is the sum of Q over the cells now; bnd_in the net inflow through
   * the domain boundary and exch the exchange total, both accumulated since
   * mm_init_state with each stage weighted by its share of the step, so that
   * sum_Q(now) - sum_Q(init) = bnd_in + exch up to rounding.  Partial sums
   * are combined in a fixed order: repeated runs give identical values. */
  double sum_Q[MM_MAX_MAT][4];
  double bnd_in[MM_MAX_MAT][4];
  double exch[MM_MAX_MAT][4];
  /* Sizes of the work lists of the last stage (2D; zero in the batched
   * form): cells outside the bulk (updated by the general cut-cell code),
   * queued ghost (cell, material) pairs, active 16 x 16 tiles. */
  int64_t n_band, n_ghost, n_tiles;
  /* Step (counted from 1 since mm_init_state) in which the non-physical
   * state of err_cell was found, -1 if none. */
  int64_t err_step;
  /* Mixing sources without an eligible target whose conserved quantities
   * joined another material of their cell (Sec. 2.3.2 mixing; a fragment of
   * the cell's own material first gives the cell to the material of largest
   * other volume fraction: n_relabel), and oddball cells of the scale
   * separation, since mm_init_state.  Where these act, totals are conserved
   * but the masses of single materials are not, and sum_Q - bnd_in - exch
   * differs from its initial value by the quantities moved. */
  int64_t n_absorb, n_relabel, n_oddball;
} mm_diag;

typedef struct mm_ctx mm_ctx;

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (e.g. torch.cuda.current_stream().cuda_stream) or NULL for the null
 * stream.  MM_EINVAL for an invalid configuration (dim, sizes, n_mat,
 * gamma <= 1, bc codes, rk_order, cfl <= 0). */
mm_status mm_create(const mm_config *cfg, void *hip_stream, mm_ctx **out);

/* Initial state (Sec. 2.2 / Eq. discretized_equ): phi >= 0 and chi in
 * [0, n_mat) per cell, and for every material a primitive field W that is
 * used wherever that material has a volume fraction.  Builds the cut-cell
 * geometry, applies the volume-fraction correction with masses alpha*rho,
 * and sets Q^0 = alpha U(W).  MM_EINVAL for NULL arrays; MM_ENONPHYS if a
 * state with alpha > 0 is non-physical. */
mm_status mm_init_state(mm_ctx *ctx, const double *phi, const int32_t *chi,
                        const double *W, int32_t ptr_kind);

/* Advance n_steps time steps (one step = all Runge-Kutta stages, with the
 * step size from the CFL condition of the time-n state, or the value set by
 * mm_set_dt).  record_tape = K > 0 keeps a tape for mm_adjoint_step: a
 * checkpoint of the state every K steps and the step size of every step
 * (a new tape starts unless the previous call recorded with the same K and
 * no step has been reversed since; MM_ENOTIMPL with the Roe face flux, for
 * which no adjoint is built); record_tape = 0 ends any tape.  If t_out
 * is not NULL it receives the time reached.  Synchronises the stream once
 * and returns MM_ENONPHYS if a non-physical real state appeared; err_cell
 * and err_step in the diagnostics name the cell and the step.  With the
 * guard on (mm_set_guard) and record_tape = 0, the state is then that after
 * the last step that completed, and the context can step on (for instance
 * with a smaller step size); otherwise the state is undefined. */
mm_status mm_step(mm_ctx *ctx, int32_t n_steps, int32_t record_tape,
                  double *t_out);

/* Copy out Q (required) and, if not NULL, alpha, phi and chi of the current
 * state, interior cells only, in the layouts above. */
mm_status mm_get_conserved(mm_ctx *ctx, double *Q, double *alpha,
                           double *phi, int32_t *chi, int32_t ptr_kind);

/* Diagnostics; synchronises the stream. */
mm_status mm_get_diagnostics(mm_ctx *ctx, mm_diag *out);

/* Replay a fixed step size instead of the CFL one; dt <= 0 restores CFL. */
mm_status mm_set_dt(mm_ctx *ctx, double dt);

/* Step-size schedule (Sec. 2.3: Delta t from the CFL condition; the
 * derivative of a run, and its finite-difference check, hold the step sizes
 * of a reference run fixed): the next n steps use dt[0], ..., dt[n-1] (host
 * array, copied), one per step, inside the captured step; afterwards the CFL
 * step size applies again.  A fixed step size (mm_set_dt) takes precedence
 * while set.  mm_init_state ends a schedule; n = 0 ends it now.  MM_EINVAL
 * if an entry is not positive and finite (nothing changed). */
mm_status mm_set_dt_schedule(mm_ctx *ctx, const double *dt, int32_t n);

/* Guard of plain steps (record_tape = 0): with enable != 0, each mm_step
 * call keeps the state it starts from (one copy of the state per call); if
 * a step of the call meets a non-physical state, the call goes back to that
 * copy and replays the steps that completed (bit for bit the same), and
 * returns MM_ENONPHYS with the state after the last completed step. */
mm_status mm_set_guard(mm_ctx *ctx, int32_t enable);

/* Differentiation (Sec. 2.3, Eq. discretized_equ, Eq. local-advection; the
 * method's step, transposed).  Reverses the last recorded step that has not
 * been reversed yet: given the adjoint of the state after it (dJ/dQ
 * [n_mat][dim+2][ny][nx], dJ/dphi [ny][nx], and dJ/dalpha [n_mat][ny][nx]
 * of its volume fractions), produce the adjoint of the state before it.
 * The step is linearised about the recorded trajectory with its step size
 * held fixed and every branch (upwind choices, HLLC wave pattern, ghost
 * sources, interface pairs, mixing sources and targets, level-set argmax,
 * volume-fraction correction) as the forward step took it.  A NULL lamQ_in
 * or lamPhi_in continues from the adjoint left by the previous call (zero
 * on the first); lamAlpha_in may be NULL.  lamQ_out / lamPhi_out may be
 * NULL.  The segment of the tape that holds the step is recomputed from
 * its checkpoint when first needed.  The forward state after the recorded
 * run and the diagnostics are left as they were.  Pointers are host or
 * device per ptr_kind.  MM_ESTATE without a recorded step to reverse.
 * Synchronises the stream when host outputs are requested; otherwise the
 * work is queued on the context's stream (host input arrays are copied
 * before the call returns). */
mm_status mm_adjoint_step(mm_ctx *ctx, const double *lamQ_in,
                          const double *lamPhi_in, const double *lamAlpha_in,
                          double *lamQ_out, double *lamPhi_out,
                          int32_t ptr_kind);

/* Adjoint of the inflow state (rho, u, v, p) collected by the reverse steps
 * taken since the tape's last step (host array of 4). */
mm_status mm_adjoint_inflow(mm_ctx *ctx, double *out);

/* Steps on the tape, steps still to reverse, and (dt not NULL, host array
 * of `recorded` entries) the recorded step sizes. */
mm_status mm_tape_info(mm_ctx *ctx, int64_t *recorded, int64_t *remaining,
                       double *dt);

/* Measurement of the dominant kernel.  With profiling enabled, every launch
 * of the bulk flux/update kernel (cells away from interfaces) is bracketed
 * by HIP events on the context's stream; mm_get_profile synchronises and
 * returns the summed kernel time, the number of launches, and the
 * algorithmic HBM bytes those launches had to move (per bulk update: read
 * Q^(s), write Q^(s+1), and read Q^n in every stage but the first; 8-byte
 * words of dim+2 components). */
typedef struct {
  double bulk_ms;          /* summed duration of the bulk launches          */
  int64_t bulk_launches;
  int64_t bulk_updates;    /* material-cell updates done by those launches  */
  double bulk_bytes;       /* algorithmic bytes of those updates            */
} mm_profile;
mm_status mm_set_profiling(mm_ctx *ctx, int32_t enable);
mm_status mm_get_profile(mm_ctx *ctx, mm_profile *out);

/* ---- Multiresolution analysis (Sec. 2.4) ------------------------------
 * The block structure the paper's adaptive grid would give the current 2D
 * state.  Levels l = 0 (coarsest) .. L (the context's grid); level l has
 * nx / 2^(L-l) x ny / 2^(L-l) cells in blocks of `block` x `block` cells, so
 * nx and ny must be multiples of block * 2^L.  Fields: the mixture density
 * and total energy (sums over the materials).  Projection: the mean of the
 * four children; prediction: the tensor product of the 1D 5th-order
 * operator u +- sum_m g_m (u[i+m] - u[i-m]), g = (-22/128, 3/128), edge
 * cells repeated beyond the domain; a detail (value - prediction) of level
 * l is significant when its magnitude exceeds 2^(2 (l - L)) eps times the
 * field's largest magnitude.  Interface position identifier: a block of the
 * context's grid with a cell whose level-set value is below `band` (the
 * narrow band), and its ancestors.  A level-l block (l < L) is refined when
 * it has the identifier or a block of its 3 x 3 neighbourhood has a
 * significant detail among its children; grading refines the parents of
 * the 3 x 3 neighbourhood of every refined block; blocks exist at level 0
 * and below refined existing blocks.
 * leaf_level: int32 per block of the context's grid ((ny/block) x
 * (nx/block), row-major): the level of the leaf covering it.  flags (NULL
 * to skip): uint8 per block, the detail flags of levels 0 .. L-1, then the
 * identifiers of levels 0 .. L, each level row-major.  Both in host or
 * device memory per ptr_kind (caller-owned); *res on the host.  MM_EINVAL
 * for a 1D context, a grid that does not divide, block < 2, L outside
 * [1, MM_MR_MAXL] or eps <= 0; MM_ESTATE before mm_init_state.  The state
 * is not changed. */
#define MM_MR_MAXL 10
typedef struct {
  int32_t block, levels;   /* block side in cells (16), L                   */
  double eps;              /* threshold of the finest level's details       */
  double band;             /* narrow band: level-set values below it        */
} mm_mr_params;
typedef struct {
  int64_t exist[MM_MR_MAXL + 1];  /* blocks that exist, per level           */
  int64_t leaf[MM_MR_MAXL + 1];   /* leaf blocks, per level                 */
  double compression;             /* leaf cells / the context's cells       */
  double scale[2];                /* largest |rho|, |rho E| (mixture)       */
} mm_mr_result;
mm_status mm_mr_analyse(mm_ctx *ctx, const mm_mr_params *p, int32_t *leaf_level,
                        uint8_t *flags, mm_mr_result *res, int32_t ptr_kind);

/* ---- Batched form ------------------------------------------------------
 * Many independent 1D problems of uneven size (same n_mat and rk_order)
 * advanced together: one persistent launch, one workgroup per instance,
 * each instance with its own step size, EOS and boundaries; the launch is
 * replayed from a HIP graph.  Arrays are the concatenation of the
 * instances' interior cells in instance order: phi, chi [sum nx]; instance
 * q's W and Q blocks are [n_mat][3][nx_q] starting at n_mat*3*off_q
 * doubles, alpha [n_mat][nx_q] at n_mat*off_q, with off_q the sum of the
 * nx of the instances before q.  Results are identical, bit for bit, to
 * advancing each instance alone with mm_step. */
typedef struct mm_batch mm_batch;
mm_status mm_batch_create(const mm_config *cfgs, int32_t n_inst, void *hip_stream,
                          mm_batch **out);
mm_status mm_batch_init_state(mm_batch *b, const double *phi, const int32_t *chi,
                              const double *W, int32_t ptr_kind);
/* Advance every instance n_steps steps; synchronises and returns
 * MM_ENONPHYS if any instance met a non-physical state.  The first call
 * chooses the workgroup size by timing candidates on a snapshot of the state
 * (restored afterwards) unless mm_batch_set_threads fixed it. */
mm_status mm_batch_step(mm_batch *b, int32_t n_steps);
mm_status mm_batch_get_conserved(mm_batch *b, double *Q, double *alpha, double *phi,
                                 int32_t *chi, int32_t ptr_kind);
/* out has n_inst entries. */
mm_status mm_batch_get_diagnostics(mm_batch *b, mm_diag *out);
/* threads: 64, 128, 256, 512 or 1024, or 0 to choose by measurement. */
mm_status mm_batch_set_threads(mm_batch *b, int32_t threads);
/* Chosen workgroup size and, if tune_ms is not NULL, the 5 trial timings
 * (64 .. 1024 threads) of the last tuning. */
mm_status mm_batch_get_threads(mm_batch *b, int32_t *threads, float *tune_ms);
mm_status mm_batch_destroy(mm_batch *b);
const char *mm_batch_last_error(const mm_batch *b);

/* ---- Batched run without device allocation ------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one call
 * initialises n_inst 1D instances from (phi, chi, W) as mm_batch_init_state
 * does, advances them n_steps steps with the kernel of mm_batch_step
 * (workgroup size `threads`: 64, 128, 256, 512 or 1024; 0 = 256; no
 * tuning), and writes the final state to Q (required), alpha, phi_out and
 * chi_out (nullable) in mm_batch_get_conserved's layout.  Every pointer is
 * device memory of the current device; results are bitwise those of
 * mm_batch_create / mm_batch_init_state / mm_batch_set_threads(threads) /
 * mm_batch_step / mm_batch_get_conserved.  All work buffers live in one
 * fixed device array of MM_NOALLOC_BYTES per GPU, held until the process
 * ends: no hipMalloc or hipFree is called.  MM_EINVAL (nothing run) if
 * n_inst exceeds MM_NOALLOC_MAX_INST or the instances need more than that
 * array; MM_ENONPHYS if an instance met a non-physical state.  Every call
 * on a GPU shares that GPU's array and clears it first: calls that overlap
 * on one GPU (other threads or streams) race.  Synchronises hip_stream
 * (NULL = the null stream).  mm_last_error(NULL) gives the message. */
#define MM_NOALLOC_BYTES (64u << 20)
#define MM_NOALLOC_MAX_INST 64
mm_status mm_batch_run_noalloc(const mm_config *cfgs, int32_t n_inst, void *hip_stream,
                               const double *phi, const int32_t *chi, const double *W,
                               int32_t n_steps, int32_t threads, double *Q, double *alpha,
                               double *phi_out, int32_t *chi_out);

/* Release every device buffer of the context. */
mm_status mm_destroy(mm_ctx *ctx);

/* Message of the last failure on ctx (thread-unsafe; valid until the next
 * call on ctx).  NULL ctx gives the last mm_create failure. */
const char *mm_last_error(const mm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MMFV_H */
