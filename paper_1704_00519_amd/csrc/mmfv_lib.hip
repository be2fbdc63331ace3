// Host side of the C ABI declared in include/mmfv.h: context, device
// buffers, and the fixed order of kernels in one time step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mmfv.h"
#include "mmfv_adjoint.h"
#include "mmfv_kernels.h"
#include "mmfv_mr.h"

using namespace mmfv;

struct mm_ctx {
  mm_config cfg;
  Params P;
  Bufs B;
  hipStream_t stream = nullptr;
  int D = 2;
  uint32_t stamp = 1;
  bool ready = false;
  int64_t steps = 0;
  std::string err;
  std::vector<void*> allocs;
  double* d_in = nullptr;   // staging of host inputs/outputs
  size_t d_in_bytes = 0;
  bool profiling = false;
  hipGraph_t step_g = nullptr;      // one captured time step
  hipGraphExec_t step_x = nullptr;
  bool graph_off = false;
  std::vector<hipEvent_t> ev;  // pairs around bulk launches
  bool bulk_wide = false;      // 28 x 32 bulk tiles (large grids)
  // after a reverse call: the counters, scalars and sums equal their saved
  // copies (until another entry point runs), and the forward tile list is
  // to be rebuilt before it is next needed
  bool adj_clean = false;
  bool tiles_stale = false;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  unsigned long long prof_u0 = 0, prof_u1 = 0;  // counters at enable time
  // tape of recorded steps for the adjoint: a checkpoint every tape_K steps
  // and the step size of every step; tape_rev steps are still to reverse
  int tape_K = 0;
  // a recorded step moved conserved quantities between materials (stranded
  // mixing sources, scale separation): the tape cannot be reversed
  bool tape_moved = false;
  int64_t tape_n = 0, tape_rev = 0;
  std::vector<char*> ckpt;
  double* tape_dt = nullptr;
  size_t tape_dt_cap = 0;
  char* seg = nullptr;  // stage snapshots of the recomputed segment
  size_t seg_cap = 0;
  int64_t seg_n0 = -1, seg_n1 = -1;
  char* final_snap = nullptr;  // state after the last recorded step
  size_t final_cap = 0;
  bool adj_ready = false;
  Adj A;
  unsigned long long* ctr_save = nullptr;
  double* scal_save = nullptr;
  double* cons_save = nullptr;
  // step-size schedule (mm_set_dt_schedule)
  double* dts = nullptr;
  size_t dts_cap = 0;
  // with the guard on, each plain mm_step call keeps the state it starts
  // from; a failing call goes back to it and replays the completed steps
  bool guard = false;
  char* guard_snap = nullptr;
  size_t guard_cap = 0;
  unsigned long long* guard_ctr = nullptr;
  double* guard_scal = nullptr;
  double* guard_cons = nullptr;
  int64_t err_step = -1;   // failing step (1-based) of the last failure
  int64_t err_cell = -1;   // its lowest non-physical cell
  // multiresolution analysis: pyramid of the two fields, flags, counts
  char* mr_buf = nullptr;
  size_t mr_cap = 0;
};

static void prof_mark(mm_ctx* c) {
  if (!c->profiling) return;
  if (c->ev_used == c->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    c->ev.push_back(e);
  }
  (void)hipEventRecord(c->ev[c->ev_used++], c->stream);
}

// sum the recorded pairs and recycle the events
static void prof_collect(mm_ctx* c) {
  if (c->ev_used < 2) return;
  (void)hipEventSynchronize(c->ev[c->ev_used - 1]);
  for (size_t q = 0; q + 1 < c->ev_used; q += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[q], c->ev[q + 1]) == hipSuccess) c->prof_ms += ms;
    c->prof_launches++;
  }
  c->ev_used = 0;
}

static std::string g_create_err;

static mm_status fail(mm_ctx* c, mm_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return s;
}

#define HIP_OK(ctx, call)                                                   \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(ctx, MM_EDEVICE, std::string(#call) + ": " +              \
                                       hipGetErrorString(e_));              \
  } while (0)

template <typename T>
static hipError_t dalloc(mm_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T) ? n * sizeof(T) : 1);
  if (e != hipSuccess) return e;
  e = hipMemset(q, 0, n * sizeof(T) ? n * sizeof(T) : 1);
  c->allocs.push_back(q);
  *p = (T*)q;
  return e;
}

static void free_all(mm_ctx* c) {
  if (c->step_x) (void)hipGraphExecDestroy(c->step_x);
  if (c->step_g) (void)hipGraphDestroy(c->step_g);
  c->step_x = nullptr;
  c->step_g = nullptr;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  for (char* p : c->ckpt) (void)hipFree(p);
  c->ckpt.clear();
  void* extra[] = {c->tape_dt, c->seg, c->final_snap, c->dts, c->guard_snap, c->guard_ctr,
                   c->guard_scal, c->guard_cons, c->mr_buf};
  for (void* p : extra)
    if (p) (void)hipFree(p);
  c->tape_dt = nullptr;
  c->seg = nullptr;
  c->final_snap = nullptr;
  c->dts = nullptr;
  c->guard_snap = nullptr;
  c->mr_buf = nullptr;
  c->mr_cap = 0;
  c->guard_ctr = nullptr;
  c->guard_scal = nullptr;
  c->guard_cons = nullptr;
  c->adj_ready = false;
  if (c->d_in) (void)hipFree(c->d_in);
  c->d_in = nullptr;
}

extern "C" const char* mm_last_error(const mm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

static bool valid_config(const mm_config* c, std::string& why) {
  if (c->dim != 1 && c->dim != 2) return why = "dim must be 1 or 2", false;
  if (c->nx < 1 || c->ny < 1) return why = "nx, ny must be >= 1", false;
  if (c->dim == 1 && c->ny != 1) return why = "ny must be 1 in 1D", false;
  if (c->n_mat < 1 || c->n_mat > MM_MAX_MAT) return why = "n_mat out of range", false;
  if (!(c->x1 > c->x0) || (c->dim == 2 && !(c->y1 > c->y0)))
    return why = "empty domain", false;
  for (int m = 0; m < c->n_mat; m++) {
    if (!(c->gamma[m] > 1.0) || !(c->pinf[m] >= 0.0))
      return why = "gamma must exceed 1 and p_inf be >= 0", false;
    if (c->eos[m] != MM_EOS_STIFFENED && c->eos[m] != MM_EOS_TAIT)
      return why = "bad eos code", false;
    if (c->eos[m] == MM_EOS_TAIT && !(c->rho0[m] > 0.0 && c->tait_B[m] > 0.0 &&
                                       std::isfinite(c->p0[m]) && c->tait_B[m] - c->p0[m] >= 0.0))
      return why = "Tait material needs rho0 > 0, B > 0 and B >= p0", false;
  }
  if (c->flux != MM_FLUX_HLLC && c->flux != MM_FLUX_ROE) return why = "bad flux code", false;
  if (c->scale_sep != 0 && c->scale_sep != 1) return why = "scale_sep must be 0 or 1", false;
  if (c->flux == MM_FLUX_ROE)
    for (int m = 0; m < c->n_mat; m++)
      if (c->eos[m] == MM_EOS_TAIT) return why = "the Roe flux takes stiffened gases only", false;
  if (c->coord != 0 && c->coord != 1) return why = "coord must be 0 or 1", false;
  if (c->coord == 1 && (c->dim != 1 || !(c->x0 >= 0.0)))
    return why = "cylindrical geometry needs dim 1 and x0 >= 0", false;
  if (c->fs_on != 0 && c->fs_on != 1) return why = "fs_on must be 0 or 1", false;
  if (c->reinit != 0 && c->reinit != 1) return why = "reinit must be 0 or 1", false;
  if (c->reinit && (c->dim != 2 || c->band_ls > 10))
    return why = "the redistancing is built for dim 2 with band_ls <= 10", false;
  if (c->fs_on) {
    if (c->dim != 1) return why = "free surfaces are built for dim 1", false;
    if (c->fs_mat < 0 || c->fs_mat >= c->n_mat) return why = "bad fs_mat", false;
    if (!(c->fs_p[4] > 0.0) || !(c->fs_p[3] > c->fs_p[2]) || !std::isfinite(c->fs_p[0]) ||
        !std::isfinite(c->fs_p[1]) || !std::isfinite(c->fs_p[3]))
      return why = "free surface needs a finite p(t), t1 > t0 and an ambient density > 0", false;
    if (c->flux != MM_FLUX_HLLC) return why = "free surfaces take the HLLC flux only", false;
    for (int m = 0; m < c->n_mat; m++)
      if (c->eos[m] == MM_EOS_TAIT) return why = "free surfaces take stiffened gases only", false;
  }
  for (int q = 0; q < 4; q++)
    if (c->bc[q] < 0 || c->bc[q] > 3) return why = "bad boundary code", false;
  if (c->inflow_mat < 0 || c->inflow_mat >= c->n_mat) return why = "bad inflow_mat", false;
  if (c->rk_order != 2 && c->rk_order != 3) return why = "rk_order must be 2 or 3", false;
  if (!(c->cfl > 0.0)) return why = "cfl must be positive", false;
  if (!(c->alpha_mix >= 0.0 && c->alpha_mix <= 1.0)) return why = "alpha_mix out of range", false;
  if (c->k_ext < 0 || c->k_ext > 8) return why = "k_ext must be in [0, 8]", false;
  if (c->band_ls < 1 || c->band_ls > 64) return why = "band_ls out of range", false;
  if ((int64_t)(c->nx + 2 * H) * (c->dim == 2 ? c->ny + 2 * H : 1) > (int64_t)1 << 31)
    return why = "grid too large", false;
  return true;
}

// workgroups of the book-keeping partial sums: boundary rows and columns
// (256 per workgroup), then cells (CONS_CH per workgroup)
static int cons_bnd_blocks(const Params& P) {
  int n = P.dim == 2 ? P.nx + P.ny : 1;
  return (n + CONS_ROWS - 1) / CONS_ROWS;
}
static int cons_cell_blocks(const Params& P) {
  return (int)(((long)P.nx * P.ny + CONS_CH - 1) / CONS_CH);
}
static int cons_blocks(const Params& P) { return cons_bnd_blocks(P) + cons_cell_blocks(P); }

static Params make_params(const mm_config* cfg) {
  Params P;
  memset(&P, 0, sizeof(P));
  P.dim = cfg->dim;
  P.nx = cfg->nx;
  P.ny = cfg->ny;
  P.NX = cfg->nx + 2 * H;
  P.HY = cfg->dim == 2 ? H : 0;
  P.NY = cfg->ny + 2 * P.HY;
  P.NC = P.NX * P.NY;
  P.M = cfg->n_mat;
  P.dx = (cfg->x1 - cfg->x0) / cfg->nx;
  P.dy = cfg->dim == 2 ? (cfg->y1 - cfg->y0) / cfg->ny : 1.0;
  P.h = cfg->dim == 2 ? (P.dx < P.dy ? P.dx : P.dy) : P.dx;
  P.bls = cfg->band_ls * P.h;
  P.idx = 1.0 / P.dx;
  P.idy = 1.0 / P.dy;
  P.amix = cfg->alpha_mix;
  P.kext = cfg->k_ext;
  P.cfl = cfg->cfl;
  for (int m = 0; m < P.M; m++) {
    P.gamma[m] = cfg->gamma[m];
    P.tait[m] = cfg->eos[m] == MM_EOS_TAIT ? 1 : 0;
    P.taitB[m] = cfg->tait_B[m];
    P.rho0[m] = cfg->rho0[m];
    P.pinf[m] = P.tait[m] ? cfg->tait_B[m] - cfg->p0[m] : cfg->pinf[m];
    P.igm1[m] = 1.0 / (cfg->gamma[m] - 1.0);
  }
  P.flux = cfg->flux == MM_FLUX_ROE ? FLUX_ROE : FLUX_HLLC;
  P.scale_sep = cfg->scale_sep;
  P.coord = cfg->coord;
  P.fs_on = cfg->fs_on;
  P.fs_mat = cfg->fs_mat;
  P.x0 = cfg->x0;
  for (int q = 0; q < 5; q++) P.fs_p[q] = cfg->fs_p[q];
  P.reinit = cfg->reinit;
  P.nband = cfg->band_ls;
  for (int q = 0; q < 4; q++) {
    P.bc[q] = cfg->bc[q];
    P.inflow_W[q] = cfg->inflow_W[q];
  }
  P.inflow_mat = cfg->inflow_mat;
  return P;
}

// workgroups of the per-cell launches (cell_grid below, from the parameters)
static dim3 cell_grid_of(const Params& P) {
  dim3 b = P.dim == 2 ? dim3(64, 4) : dim3(256, 1);
  return dim3((P.nx + b.x - 1) / b.x, (P.ny + b.y - 1) / b.y);
}

extern "C" mm_status mm_create(const mm_config* cfg, void* hip_stream, mm_ctx** out) {
  if (!cfg || !out) return fail(nullptr, MM_EINVAL, "NULL argument");
  std::string why;
  if (!valid_config(cfg, why)) return fail(nullptr, MM_EINVAL, why);
  mm_ctx* c = new mm_ctx();
  c->cfg = *cfg;
  c->D = cfg->dim;
  c->stream = (hipStream_t)hip_stream;
  c->P = make_params(cfg);
  const Params& P = c->P;
  {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    long tiles = (long)((P.nx + BULK_BX - 1) / BULK_BX) * ((P.ny + BULK_BY - 1) / BULK_BY);
    c->bulk_wide = P.dim == 2 && tiles > (long)BULK_WIDE_TILES_PER_CU * (cus > 0 ? cus : 256);
    (void)hipGetLastError();
  }

  size_t nc = P.NC, M = P.M, nv = P.dim + 2;
  Bufs& B = c->B;
  memset(&B, 0, sizeof(B));
  hipError_t e = hipSuccess;
#define A(p, n)                               \
  if (e == hipSuccess) e = dalloc(c, &(p), (n));
  for (int b = 0; b < 3; b++) {
    A(B.Q[b], M * nv * nc);
    A(B.occ[b], (nc + 255) & ~(size_t)255);  // whole 32-bit words for word atomics
  }
  A(B.phi, nc); A(B.ptmp, nc); A(B.phin, nc);
  A(B.chi, nc); A(B.ctmp, nc); A(B.chin, nc);
  A(B.al, M * nc); A(B.ax, M * nc); A(B.ay, M * nc); A(B.cx, M * nc); A(B.cy, M * nc);
  A(B.W, M * 4 * nc); A(B.Wit, M * nc);
  A(B.cut, nc); A(B.xs, nc); A(B.dcut, nc); A(B.dls, nc); A(B.rowc, nc); A(B.rowl, nc);
  A(B.tdc, nc); A(B.tdl, nc);
  A(B.nrow, nc); A(B.near4, nc); A(B.bulk, nc);
  A(B.X, M * 4 * nc);
  A(B.vx, nc); A(B.vy, nc); A(B.vit, nc);
  A(B.mixM, M * 3 * 4 * nc); A(B.mixT, M * 3 * nc);
  A(B.srcStamp, M * nc); A(B.tgtStamp, M * nc);
  {
    size_t ncb = (size_t)((P.nx + CX - 1) / CX) * ((P.ny + CY - 1) / CY);
    A(B.cquiet[0], ncb); A(B.cquiet[1], ncb);
  }
  A(B.strStamp, M * nc); A(B.abMark, nc); A(B.rlStamp, nc);
  A(B.rlTo, nc); A(B.ssTo, nc); A(B.abList, nc); A(B.ssList, nc); A(B.ssPhi, nc);
  A(B.tiles, (size_t)((P.nx + 15) / 16 + 16) * ((P.ny + 15) / 16 + 1));
  A(B.blist, nc);
  A(B.glist, M * nc);
  A(B.scal, 8); A(B.ctr, C_N);
  A(B.vfc, nc);
  A(B.cons, CONS_N);
  {
    dim3 gb = cell_grid_of(P);
    A(B.dtpart, (size_t)gb.x * gb.y);
  }
  A(B.cpart, (size_t)cons_blocks(P) * M * 8);
#undef A
  if (e != hipSuccess) {
    free_all(c);
    delete c;
    return fail(nullptr, e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EDEVICE,
                std::string("allocation: ") + hipGetErrorString(e));
  }
  unsigned long long init_ctr[C_N] = {0};
  init_ctr[C_ERR] = NO_ERR;
  init_ctr[C_ERRSTEP] = NO_ERR;
  init_ctr[C_STAMP] = 1;
  if (hipMemcpy(B.ctr, init_ctr, sizeof(init_ctr), hipMemcpyHostToDevice) != hipSuccess) {
    free_all(c);
    delete c;
    return fail(nullptr, MM_EDEVICE, "counter init");
  }
  *out = c;
  return MM_OK;
}

extern "C" mm_status mm_destroy(mm_ctx* c) {
  if (!c) return MM_EINVAL;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_all(c);
  delete c;
  return MM_OK;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static dim3 cell_block(const mm_ctx* c) { return c->D == 2 ? dim3(64, 4) : dim3(256, 1); }
static dim3 cell_grid(const mm_ctx* c) {
  dim3 b = cell_block(c);
  return dim3((c->P.nx + b.x - 1) / b.x, (c->P.ny + b.y - 1) / b.y);
}
static dim3 lin_grid(long n) { return dim3((unsigned)((n + 255) / 256)); }

#define LAUNCH(kern, grid, block, ...) \
  hipLaunchKernelGGL(kern, grid, block, 0, c->stream, __VA_ARGS__)

// Several device-to-device copies (and fills) in one launch (grid y = entry
// index)
__global__ void __launch_bounds__(256) k_copy_multi(CopyList L) {
  int e = blockIdx.y;
  if (e >= L.n) return;
  size_t words = L.bytes[e] / 8, tail = L.bytes[e] % 8;
  const double* s8 = (const double*)L.src[e];
  double* d8 = (double*)L.dst[e];
  bool fill = s8 == nullptr;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
       w += (size_t)gridDim.x * blockDim.x)
    d8[w] = fill ? 0.0 : s8[w];
  if (blockIdx.x == 0 && threadIdx.x < tail)
    L.dst[e][words * 8 + threadIdx.x] = fill ? 0 : L.src[e][words * 8 + threadIdx.x];
}
struct Copies {
  // entries of one batch are independent: a full list is launched on its own
  std::vector<std::pair<CopyList, size_t>> full;
  CopyList L;
  size_t maxw = 0;
  Copies() { L.n = 0; }
  void add(void* dst, const void* src, size_t bytes) {
    if (L.n == MAXCOPY) {
      full.emplace_back(L, maxw);
      L.n = 0;
      maxw = 0;
    }
    L.src[L.n] = (const char*)src;
    L.dst[L.n] = (char*)dst;
    L.bytes[L.n] = bytes;
    L.n++;
    if (bytes / 8 > maxw) maxw = bytes / 8;
  }
  void fill0(void* dst, size_t bytes) { add(dst, nullptr, bytes); }
  static void launch(mm_ctx* c, const CopyList& l, size_t mw) {
    unsigned gx = (unsigned)((mw + 255) / 256);
    if (gx > 512) gx = 512;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_copy_multi, dim3(gx, l.n), dim3(256), 0, c->stream, l);
  }
  void run(mm_ctx* c) {
    for (auto& f : full) launch(c, f.first, f.second);
    full.clear();
    if (L.n) launch(c, L, maxw);
    L.n = 0;
    maxw = 0;
  }
};



template <int D>
static void bc_ls(mm_ctx* c) {
  const Params& P = c->P;
  LAUNCH(k_bc_ls_x, lin_grid((long)P.ny * 2 * H), dim3(256), P, c->B, c->B.phi, c->B.chi);
  if (D == 2)
    LAUNCH(k_bc_ls_y, lin_grid((long)(P.nx + 2 * H) * 2 * H), dim3(256), P, c->B, c->B.phi,
           c->B.chi);
}

// gate >= 0: the launches run only when counter gate holds the stage's stamp
template <int D>
static void classify(mm_ctx* c, int gate = -1) {
  const Params& P = c->P;
  if (D == 2) {
    LAUNCH(k_classify_dist2, dim3((P.nx + CX - 1) / CX, (P.ny + CY - 1) / CY), dim3(256), P,
           c->B, gate);
  } else {
    LAUNCH(k_classify<D>, cell_grid(c), cell_block(c), P, c->B, gate);
    LAUNCH(k_dist_row<D>, cell_grid(c), cell_block(c), P, c->B, gate);
  }
}

static int n_tiles(const Params& P) {
  int tw = P.dim == 2 ? 16 : 256, th = P.dim == 2 ? 16 : 1;
  return ((P.nx + tw - 1) / tw) * ((P.ny + th - 1) / th);
}
static dim3 tile_grid(const mm_ctx* c) {
  int n = n_tiles(c->P);
  return dim3(n < 1024 ? n : 1024);
}

// list the active tiles after the level set of the next stage is known
template <int D>
static void build_tiles(mm_ctx* c, int didx, int nidx) {
  LAUNCH(k_tiles, dim3(n_tiles(c->P)), dim3(256), c->P, c->B, didx, nidx);
}

// the forward tile list after reverse calls emptied it
static void ensure_tiles(mm_ctx* c) {
  if (!c->tiles_stale) return;
  Copies z;
  z.fill0(&c->B.ctr[C_NTILES], sizeof(unsigned long long));
  z.run(c);
  if (c->D == 2) build_tiles<2>(c, 0, 0);
  else build_tiles<1>(c, 0, 0);
  c->tiles_stale = false;
}

// first half of a stage: real and ghost states, interface exchange (and at
// stage 0 the level-set velocity and dt), fluxes and the RK update into
// buffer didx beside the level-set stage, conservation book-keeping
// partials (in 1D also the totals and, with advance, the time)
template <int D>
static void stage_fluid(mm_ctx* c, int s, int sidx, int nidx, int didx, double b, double cc,
                        double w, bool advance, const CopyList& pre) {
  const Params& P = c->P;
  dim3 g = cell_grid(c), bl = cell_block(c);
  dim3 tg = tile_grid(c), tb(256);
  LAUNCH(t_real_near_row<D>, dim3(2 * tg.x + (pre.n ? 256 : 0)), tb, P, c->B, sidx, (int)tg.x,
         pre);
  // the ambient of a free surface: its prescribed state and conserved
  // quantities at the stage's time (before the ghost queue and the bulk
  // flags, which read its validity and occupancy)
  if (P.fs_on) LAUNCH(k_ambient<D>, lin_grid(P.NC), dim3(256), P, c->B, sidx, s);
  LAUNCH(t_near_col_flags<D>, dim3(tg.x + g.x * g.y), tb, P, c->B, sidx, nidx, s == 0 ? 1 : 0,
         (int)tg.x, (int)g.x, (int)g.y, (int)bl.x);
  static_assert(EXR >= 8 + 4, "the tile frame covers every sweep (k_ext <= 8)");
  if (D == 2) {
    LAUNCH(k_ext_tiles, dim3(tg.x, P.M), tb, P, c->B, sidx);
  } else {
    // the sweeps of a 1D stage in one workgroup (its queue is short)
    LAUNCH(k_ext_all1, dim3(1), dim3(1024), P, c->B, sidx);
  }
  long nframe = (D == 2 ? (long)P.ny + P.nx + 2 * H : (long)P.ny) * 2 * H * P.M;
  int ndt = s == 0 ? (int)(g.x * g.y) : 0;  // stage 0: one more workgroup sets the step size
  LAUNCH(t_iface_frame<D>, dim3(tg.x + lin_grid(nframe).x + (ndt ? 1 : 0)), tb, P, c->B, sidx,
         s, (int)tg.x, ndt);
  if (s == 0 && D == 2) {
    LAUNCH(k_vext_tiles, tg, tb, P, c->B, sidx);
  } else if (s == 0) {
    LAUNCH(k_vel_all1, dim3(1), dim3(1024), P, c->B, sidx);
  }
  prof_mark(c);
  if (D == 2 && P.flux == FLUX_ROE)
    // the characteristic projection needs more registers than the 1024-thread
    // tile leaves a thread: the 512-thread tile at any grid size
    LAUNCH((k_flux_bulk2<BULK_BX, BULK_BY, BULK_NT, FLUX_ROE>),
           dim3((P.nx + BULK_BX - 1) / BULK_BX, (P.ny + BULK_BY - 1) / BULK_BY),
           dim3(BULK_NT), P, c->B, sidx, nidx, didx, b, cc, s == 0 ? 1 : 0);
  else if (D == 2)
    if (c->bulk_wide)
      LAUNCH((k_flux_bulk2<BULK_BXW, BULK_BYW, BULK_NTW, FLUX_HLLC>),
             dim3((P.nx + BULK_BXW - 1) / BULK_BXW, (P.ny + BULK_BYW - 1) / BULK_BYW),
             dim3(BULK_NTW), P, c->B, sidx, nidx, didx, b, cc, s == 0 ? 1 : 0);
    else
      LAUNCH((k_flux_bulk2<BULK_BX, BULK_BY, BULK_NT, FLUX_HLLC>),
             dim3((P.nx + BULK_BX - 1) / BULK_BX, (P.ny + BULK_BY - 1) / BULK_BY),
             dim3(BULK_NT), P, c->B, sidx, nidx, didx, b, cc, s == 0 ? 1 : 0);
  else
    LAUNCH(k_flux_bulk1, dim3((P.nx + T1 - 1) / T1), dim3(T1), P, c->B, sidx, nidx, didx, b,
           cc, s == 0 ? 1 : 0);
  prof_mark(c);
  if (c->ev_used >= 4096) prof_collect(c);
  // band update with the book-keeping partials and the level-set stage
  constexpr int FLUX_LIST_BLOCKS = 2048;
  if (P.flux == FLUX_ROE)
    LAUNCH((k_flux_list_cons<D, FLUX_ROE>), dim3(cons_blocks(P) * P.M + tg.x + FLUX_LIST_BLOCKS),
           dim3(256), P, c->B, sidx, nidx, didx, b, cc, FLUX_LIST_BLOCKS, cons_bnd_blocks(P),
           cons_blocks(P), (int)tg.x);
  else
    LAUNCH((k_flux_list_cons<D, FLUX_HLLC>), dim3(cons_blocks(P) * P.M + tg.x + FLUX_LIST_BLOCKS),
           dim3(256), P, c->B, sidx, nidx, didx, b, cc, FLUX_LIST_BLOCKS, cons_bnd_blocks(P),
           cons_blocks(P), (int)tg.x);
  if (D == 1)
    LAUNCH(k_cons_fin, dim3(P.M * 8), dim3(64), P, c->B, cons_blocks(P), w, advance ? 1 : 0);
}

// second half: commit of the level-set stage (computed beside the band
// update) and its frame, with the stage's book-keeping totals in 2D (and
// with advance, the time), classification, geometry and correction of the
// new level set, mixing (with save, Q* is copied before the mixing for the
// adjoint)
template <int D>
static void stage_levelset(mm_ctx* c, int didx, int nidx, double w, bool advance,
                           double* save_Q, uint8_t* save_occ, const CopyList& post) {
  const Params& P = c->P;
  dim3 tg = tile_grid(c), tb(256);
  if (D == 2) {
    long nframe = ((long)P.ny + P.nx + 2 * H) * 2 * H;
    unsigned nfr = (unsigned)((nframe + 255) / 256), nfin = (unsigned)(P.M * 8 + 3) / 4;
    LAUNCH(k_ls_commit_bc, dim3(tg.x + nfr + nfin), tb, P, c->B, (int)tg.x, (int)nfr,
           cons_blocks(P), w, advance ? 1 : 0);
  } else {
    LAUNCH(t_ls_commit<D>, tg, tb, P, c->B);
    bc_ls<D>(c);
  }
  classify<D>(c);
  int nt = n_tiles(P);
  // with save_Q, Q* and its occupancy are copied by extra workgroups
  int nb = nt;  // one workgroup per tile and part (measured faster than fewer, longer ones)
  LAUNCH(k_tiles_geom<D>, dim3(2 * nb + (save_Q ? 512 : 0)), tb, P, c->B, didx, nidx, nt, nb,
         save_Q, save_occ, -1);
  LAUNCH(t_mix1<D>, dim3(tg.x, P.M), tb, P, c->B, didx);
  LAUNCH(t_mix2<D>, dim3(tg.x, P.M, post.n ? 2 : 1), tb, P, c->B, didx, post);
  // stranded sources; where a cell was relabelled, classification and
  // geometry once more (these launches return at once otherwise)
  LAUNCH(k_absorb<D>, dim3(1), tb, P, c->B, didx);
  classify<D>(c, C_RLSTAMP);
  LAUNCH(k_tiles_geom<D>, dim3(2 * nb), tb, P, c->B, didx, nidx, nt, nb, (double*)nullptr,
         (uint8_t*)nullptr, (int)C_RLSTAMP);
}

// scale separation after a step: oddball cells of the listed tiles, their
// swap, then classification and geometry once more if there was one
template <int D>
static void scale_separation(mm_ctx* c) {
  const Params& P = c->P;
  dim3 tg = tile_grid(c), tb(256);
  int nt = n_tiles(P);
  LAUNCH(t_ss_detect<D>, tg, tb, P, c->B);
  LAUNCH(k_ss_apply<D>, dim3(1), tb, P, c->B, 0);
  classify<D>(c, C_SSSTAMP);
  LAUNCH(k_tiles_geom<D>, dim3(2 * nt), tb, P, c->B, 0, 0, nt, nt, (double*)nullptr,
         (uint8_t*)nullptr, (int)C_SSSTAMP);
}

// pre / post: copies run by extra workgroups of the stage's first and last
// launches (the adjoint's recompute), none for a plain step
static const CopyList kNoCopies = {{}, {}, {}, 0};
template <int D>
static void stage(mm_ctx* c, int s, int sidx, int nidx, int didx, double b, double cc,
                  double w, double* save_Q = nullptr, uint8_t* save_occ = nullptr,
                  bool advance = false, const CopyList& pre = kNoCopies,
                  const CopyList& post = kNoCopies) {
  stage_fluid<D>(c, s, sidx, nidx, didx, b, cc, w, advance, pre);
  stage_levelset<D>(c, didx, nidx, w, advance, save_Q, save_occ, post);
}

// beta-form coefficients, and each stage's share w of the full step in the
// final combination (used by the conservation book-keeping)
static int rk_coefs(const mm_config& cfg, double* b, double* cc, double* w) {
  if (cfg.rk_order == 2) {
    b[0] = 0.0; b[1] = 0.5;
    cc[0] = 1.0; cc[1] = 0.5;
    w[0] = 0.5; w[1] = 0.5;
    return 2;
  }
  b[0] = 0.0; b[1] = 0.75; b[2] = 1.0 / 3.0;
  cc[0] = 1.0; cc[1] = 0.25; cc[2] = 2.0 / 3.0;
  w[0] = 1.0 / 6.0; w[1] = 1.0 / 6.0; w[2] = 2.0 / 3.0;
  return 3;
}
// state buffers of stage s of ns: 0 holds time n; stages write 1, 2 and
// finally 0 in place
static int stage_src(int s) { return s; }
static int stage_dst(int s, int ns) { return s == ns - 1 ? 0 : s + 1; }

// redistancing of the level set after a step (2D), then classification and
// geometry of the new level set
template <int D>
static void reinit_levelset(mm_ctx* c) {
  const Params& P = c->P;
  dim3 tg = tile_grid(c), tb(256);
  LAUNCH(k_reinit_tiles, tg, tb, P, c->B);
  LAUNCH(k_reinit_commit, tg, tb, P, c->B);
  bc_ls<D>(c);
  classify<D>(c);
  int nt = n_tiles(P);
  LAUNCH(k_tiles_geom<D>, dim3(2 * nt), tb, P, c->B, 0, 0, nt, nt, (double*)nullptr,
         (uint8_t*)nullptr, -1);
}

template <int D>
static void one_step(mm_ctx* c) {
  double b[3], cc[3], w[3];
  int ns = rk_coefs(c->cfg, b, cc, w);
  // the last stage's book-keeping also advances the time
  for (int s = 0; s < ns; s++)
    stage<D>(c, s, stage_src(s), 0, stage_dst(s, ns), b[s], cc[s], w[s], nullptr, nullptr,
             s == ns - 1);
  if (c->P.scale_sep) scale_separation<D>(c);
  if (D == 2 && c->P.reinit) reinit_levelset<D>(c);
}

static mm_status stage_inputs(mm_ctx* c, size_t bytes, const void* src, int ptr_kind,
                              const void** dev) {
  if (ptr_kind == MM_DEVICE) {
    *dev = src;
    return MM_OK;
  }
  return MM_OK;
}

extern "C" mm_status mm_init_state(mm_ctx* c, const double* phi, const int32_t* chi,
                                   const double* W, int32_t ptr_kind) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  c->tiles_stale = false;
  if (!phi || !chi || !W) return fail(c, MM_EINVAL, "NULL input array");
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return fail(c, MM_EINVAL, "bad ptr_kind");
  const Params& P = c->P;
  size_t plane = (size_t)P.nx * P.ny, nv = P.dim + 2;
  size_t nW = (size_t)P.M * nv * plane;
  const double *dphi = phi, *dW = W;
  const int32_t* dchi = chi;
  if (ptr_kind == MM_HOST) {
    for (size_t q = 0; q < plane; q++)
      if (chi[q] < 0 || chi[q] >= P.M || !(phi[q] >= 0.0))
        return fail(c, MM_EINVAL, "chi out of range or phi negative");
    size_t need = (plane + nW) * sizeof(double) + plane * sizeof(int32_t);
    if (c->d_in_bytes < need) {
      if (c->d_in) (void)hipFree(c->d_in);
      c->d_in = nullptr;
      c->d_in_bytes = 0;
      if (hipMalloc(&c->d_in, need) != hipSuccess) return fail(c, MM_ENOMEM, "staging buffer");
      c->d_in_bytes = need;
    }
    double* p0 = c->d_in;
    double* w0 = p0 + plane;
    int32_t* c0 = (int32_t*)(w0 + nW);
    HIP_OK(c, hipMemcpyAsync(p0, phi, plane * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(w0, W, nW * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(c0, chi, plane * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    dphi = p0;
    dW = w0;
    dchi = c0;
  }
  unsigned long long init_ctr[C_N] = {0};
  init_ctr[C_ERR] = NO_ERR;
  init_ctr[C_ERRSTEP] = NO_ERR;
  init_ctr[C_STAMP] = 1;
  HIP_OK(c, hipMemcpyAsync(c->B.ctr, init_ctr, sizeof(init_ctr), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemsetAsync(c->B.scal, 0, 8 * sizeof(double), c->stream));
  HIP_OK(c, hipMemsetAsync(c->B.cons, 0, CONS_N * sizeof(double), c->stream));
  for (int b = 0; b < 3; b++) HIP_OK(c, hipMemsetAsync(c->B.occ[b], 0, P.NC, c->stream));
  // stamps start again from 1: no mark of an earlier run may match
  {
    size_t nc = P.NC, M = P.M;
    HIP_OK(c, hipMemsetAsync(c->B.srcStamp, 0, M * nc * 4, c->stream));
    HIP_OK(c, hipMemsetAsync(c->B.tgtStamp, 0, M * nc * 4, c->stream));
    HIP_OK(c, hipMemsetAsync(c->B.strStamp, 0, M * nc * 4, c->stream));
    HIP_OK(c, hipMemsetAsync(c->B.abMark, 0, nc * 4, c->stream));
    HIP_OK(c, hipMemsetAsync(c->B.rlStamp, 0, nc * 4, c->stream));
    size_t ncb = (size_t)((P.nx + CX - 1) / CX) * ((P.ny + CY - 1) / CY);
    HIP_OK(c, hipMemsetAsync(c->B.cquiet[0], 0, ncb, c->stream));
    HIP_OK(c, hipMemsetAsync(c->B.cquiet[1], 0, ncb, c->stream));
  }
  dim3 g = cell_grid(c), bl = cell_block(c);
  LAUNCH(k_load_ls, g, bl, P, c->B, dphi, dchi);
  if (c->D == 2) {
    bc_ls<2>(c);
    classify<2>(c);
    LAUNCH(k_geom<2>, g, bl, P, c->B, 0, dW);
    LAUNCH(k_init_Q<2>, g, bl, P, c->B, dW);
    build_tiles<2>(c, 0, 0);
  } else {
    bc_ls<1>(c);
    classify<1>(c);
    LAUNCH(k_geom<1>, g, bl, P, c->B, 0, dW);
    LAUNCH(k_init_Q<1>, g, bl, P, c->B, dW);
    build_tiles<1>(c, 0, 0);
  }
  HIP_OK(c, hipGetLastError());
  HIP_OK(c, hipStreamSynchronize(c->stream));
  unsigned long long ctr[C_N];
  HIP_OK(c, hipMemcpy(ctr, c->B.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  c->steps = 0;
  c->ready = true;
  c->err_cell = c->err_step = -1;
  if (ctr[C_BADIN] != 0) {
    c->ready = false;
    return fail(c, MM_EINVAL, std::to_string(ctr[C_BADIN]) +
                                  " cells with chi out of range or phi negative");
  }
  if (ctr[C_ERR] != NO_ERR) {
    c->ready = false;
    return fail(c, MM_ENONPHYS, "non-physical initial state at cell " + std::to_string(ctr[C_ERR]));
  }
  (void)stage_inputs;
  return MM_OK;
}

// enqueue n time steps: one captured step replayed per time step when the
// work goes to a real stream (the null stream cannot be captured, and
// per-kernel profiling needs its events between launches), else direct
// launches
static mm_status launch_steps(mm_ctx* c, int32_t n_steps) {
  bool graph = c->stream && !c->profiling && !c->graph_off && getenv("MMFV_NO_GRAPH") == nullptr;
  if (graph && !c->step_x) {
    bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      if (c->D == 2) one_step<2>(c);
      else one_step<1>(c);
      ok = hipStreamEndCapture(c->stream, &c->step_g) == hipSuccess && c->step_g;
    }
    if (ok) ok = hipGraphInstantiate(&c->step_x, c->step_g, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      c->graph_off = true;
      graph = false;
    }
  }
  for (int n = 0; n < n_steps; n++) {
    if (graph) {
      HIP_OK(c, hipGraphLaunch(c->step_x, c->stream));
    } else if (c->D == 2) {
      one_step<2>(c);
    } else {
      one_step<1>(c);
    }
  }
  HIP_OK(c, hipGetLastError());
  c->steps += n_steps;
  return MM_OK;
}

static mm_status guard_save(mm_ctx* c);
static mm_status guard_rollback(mm_ctx* c, int64_t steps0, int64_t done);

// after a batch of steps: optional time output, then the error check (the
// one synchronisation).  With guard_from >= 0 (the step count at the start
// of a guarded call) a failure rolls back to the last completed step.
static mm_status finish_steps(mm_ctx* c, double* t_out, int64_t guard_from = -1) {
  if (t_out) {
    HIP_OK(c, hipMemcpyAsync(t_out, c->B.scal + S_T, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  unsigned long long err = 0, errstep = 0;
  HIP_OK(c, hipMemcpyAsync(&err, c->B.ctr + C_ERR, sizeof(err), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipMemcpyAsync(&errstep, c->B.ctr + C_ERRSTEP, sizeof(errstep),
                           hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (err != NO_ERR) {
    c->err_cell = (int64_t)err;
    c->err_step = errstep == NO_ERR ? -1 : (int64_t)errstep + 1;
    if (guard_from >= 0 && errstep != NO_ERR && (int64_t)errstep >= guard_from) {
      mm_status st = guard_rollback(c, guard_from, (int64_t)errstep - guard_from);
      if (st != MM_OK) return st;
      if (t_out)
        HIP_OK(c, hipMemcpy(t_out, c->B.scal + S_T, sizeof(double), hipMemcpyDeviceToHost));
      return fail(c, MM_ENONPHYS, "non-physical state at cell " + std::to_string(err) +
                                      " in step " + std::to_string(c->err_step) +
                                      "; the state after step " + std::to_string(c->steps) +
                                      " is kept");
    }
    c->ready = false;
    return fail(c, MM_ENONPHYS, "non-physical state at cell " + std::to_string(err) +
                                    " in step " + std::to_string(c->err_step));
  }
  return MM_OK;
}

static mm_status step_record(mm_ctx* c, int32_t n_steps, int32_t K, double* t_out);

extern "C" mm_status mm_step(mm_ctx* c, int32_t n_steps, int32_t record_tape, double* t_out) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  ensure_tiles(c);
  if (!c->ready) return fail(c, MM_ESTATE, "mm_step before mm_init_state");
  if (n_steps < 0) return fail(c, MM_EINVAL, "n_steps < 0");
  if (record_tape < 0) return fail(c, MM_EINVAL, "record_tape < 0");
  if (record_tape > 0 && c->P.flux != FLUX_HLLC)
    return fail(c, MM_ENOTIMPL, "the adjoint is built for the HLLC face flux only");
  if (record_tape > 0 && (c->P.coord != 0 || c->P.fs_on))
    return fail(c, MM_ENOTIMPL, "the adjoint is built for planar geometry without free surfaces");
  if (record_tape > 0 && c->P.reinit)
    return fail(c, MM_ENOTIMPL, "the adjoint is built without the level-set redistancing");
  if (record_tape > 0) return step_record(c, n_steps, record_tape, t_out);
  c->tape_K = 0;  // plain steps end any tape
  c->tape_n = c->tape_rev = 0;
  c->seg_n0 = -1;
  int64_t steps0 = c->steps;
  if (c->guard && n_steps > 0) {
    mm_status st = guard_save(c);
    if (st != MM_OK) return st;
  }
  mm_status st = launch_steps(c, n_steps);
  if (st != MM_OK) return st;
  return finish_steps(c, t_out, c->guard ? steps0 : -1);
}

extern "C" mm_status mm_get_conserved(mm_ctx* c, double* Q, double* alpha, double* phi,
                                      int32_t* chi, int32_t ptr_kind) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  if (!Q) return fail(c, MM_EINVAL, "Q must not be NULL");
  if (!c->ready && c->steps == 0) return fail(c, MM_ESTATE, "no state");
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return fail(c, MM_EINVAL, "bad ptr_kind");
  const Params& P = c->P;
  size_t plane = (size_t)P.nx * P.ny, nv = P.dim + 2;
  size_t nQ = (size_t)P.M * nv * plane, nA = (size_t)P.M * plane;
  dim3 g = cell_grid(c), bl = cell_block(c);
  if (ptr_kind == MM_DEVICE) {
    if (c->D == 2) LAUNCH(k_pack<2>, g, bl, P, c->B, 0, Q, alpha, phi, chi);
    else LAUNCH(k_pack<1>, g, bl, P, c->B, 0, Q, alpha, phi, chi);
    HIP_OK(c, hipGetLastError());
    return MM_OK;
  }
  size_t need = (nQ + nA + plane) * sizeof(double) + plane * sizeof(int32_t);
  if (c->d_in_bytes < need) {
    if (c->d_in) (void)hipFree(c->d_in);
    c->d_in = nullptr;
    c->d_in_bytes = 0;
    if (hipMalloc(&c->d_in, need) != hipSuccess) return fail(c, MM_ENOMEM, "staging buffer");
    c->d_in_bytes = need;
  }
  double* q0 = c->d_in;
  double* a0 = q0 + nQ;
  double* p0 = a0 + nA;
  int32_t* c0 = (int32_t*)(p0 + plane);
  if (c->D == 2) LAUNCH(k_pack<2>, g, bl, P, c->B, 0, q0, a0, p0, c0);
  else LAUNCH(k_pack<1>, g, bl, P, c->B, 0, q0, a0, p0, c0);
  HIP_OK(c, hipGetLastError());
  HIP_OK(c, hipMemcpyAsync(Q, q0, nQ * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (alpha)
    HIP_OK(c, hipMemcpyAsync(alpha, a0, nA * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (phi)
    HIP_OK(c, hipMemcpyAsync(phi, p0, plane * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (chi)
    HIP_OK(c, hipMemcpyAsync(chi, c0, plane * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

// copy the book-keeping of one context (or instance) into a diag record
static void cons_to_diag(const double* cons, int M, mm_diag* out) {
  memset(out->sum_Q, 0, sizeof(out->sum_Q));
  memset(out->bnd_in, 0, sizeof(out->bnd_in));
  memset(out->exch, 0, sizeof(out->exch));
  for (int r = 0; r < M; r++)
    for (int v = 0; v < 4; v++) {
      out->sum_Q[r][v] = cons[(CONS_Q * MAXM + r) * 4 + v];
      out->bnd_in[r][v] = cons[(CONS_BND * MAXM + r) * 4 + v] + cons[(CONS_BNDC * MAXM + r) * 4 + v];
      out->exch[r][v] = cons[(CONS_X * MAXM + r) * 4 + v] + cons[(CONS_XC * MAXM + r) * 4 + v];
    }
}

extern "C" mm_status mm_get_diagnostics(mm_ctx* c, mm_diag* out) {
  if (!c || !out) return MM_EINVAL;
  c->adj_clean = false;
  ensure_tiles(c);
  unsigned long long ctr[C_N];
  double scal[8];
  std::vector<double> cons(CONS_N);
  int nqb = cons_cell_blocks(c->P);
  if (c->D == 2) LAUNCH(k_qsum_part<2>, dim3(nqb), dim3(256), c->P, c->B, 0);
  else LAUNCH(k_qsum_part<1>, dim3(nqb), dim3(256), c->P, c->B, 0);
  LAUNCH(k_qsum_fin, dim3(1), dim3(256), c->P, c->B, nqb);
  HIP_OK(c, hipGetLastError());
  HIP_OK(c, hipMemcpyAsync(cons.data(), c->B.cons, CONS_N * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(ctr, c->B.ctr, sizeof(ctr), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipMemcpyAsync(scal, c->B.scal, sizeof(scal), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  out->t = scal[S_T];
  out->dt = scal[S_DT];
  out->steps = c->steps;
  out->n_posfix = (int64_t)ctr[C_POSFIX];
  out->n_fluxskip = (int64_t)ctr[C_FLUXSKIP];
  out->n_ifskip = (int64_t)ctr[C_IFSKIP];
  out->n_stranded = (int64_t)ctr[C_STRANDED];
  out->n_absorb = (int64_t)ctr[C_ABSORB];
  out->n_relabel = (int64_t)ctr[C_RELABEL];
  out->n_oddball = (int64_t)ctr[C_ODDBALL];
  out->n_mixsrc = (int64_t)ctr[C_MIXSRC];
  out->n_updates = (int64_t)ctr[C_UPD];
  out->err_cell = ctr[C_ERR] == NO_ERR ? c->err_cell : (int64_t)ctr[C_ERR];
  out->err_step = ctr[C_ERRSTEP] == NO_ERR ? c->err_step : (int64_t)ctr[C_ERRSTEP] + 1;
  out->n_band = c->D == 2 ? (int64_t)ctr[C_NBAND] : 0;
  out->n_ghost = c->D == 2 ? (int64_t)ctr[C_NGHOST] : 0;
  out->n_tiles = c->D == 2 ? (int64_t)ctr[C_NTILES] : 0;
  cons_to_diag(cons.data(), c->P.M, out);
  return MM_OK;
}

extern "C" mm_status mm_set_dt(mm_ctx* c, double dt) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  double v = dt > 0.0 ? dt : 0.0;
  HIP_OK(c, hipMemcpyAsync(c->B.scal + S_DTFIX, &v, sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

extern "C" mm_status mm_set_dt_schedule(mm_ctx* c, const double* dt, int32_t n) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  if (n < 0 || (n > 0 && !dt)) return fail(c, MM_EINVAL, "bad schedule");
  for (int32_t q = 0; q < n; q++)
    if (!(dt[q] > 0.0) || !std::isfinite(dt[q]))
      return fail(c, MM_EINVAL, "schedule entries must be positive and finite");
  if ((size_t)n > c->dts_cap) {
    // the captured step holds the buffer table by value: capture again
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double* nd = nullptr;
    HIP_OK(c, hipMalloc((void**)&nd, (size_t)n * sizeof(double)));
    if (c->dts) (void)hipFree(c->dts);
    c->dts = nd;
    c->dts_cap = (size_t)n;
    c->B.dts = nd;
    if (c->step_x) (void)hipGraphExecDestroy(c->step_x);
    if (c->step_g) (void)hipGraphDestroy(c->step_g);
    c->step_x = nullptr;
    c->step_g = nullptr;
  }
  if (n > 0)
    HIP_OK(c, hipMemcpyAsync(c->dts, dt, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
  double pos[2] = {0.0, (double)n};
  HIP_OK(c, hipMemcpyAsync(c->B.scal + S_SPOS, pos, sizeof(pos), hipMemcpyHostToDevice,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

extern "C" mm_status mm_set_guard(mm_ctx* c, int32_t enable) {
  if (!c) return MM_EINVAL;
  c->guard = enable != 0;
  return MM_OK;
}

extern "C" mm_status mm_set_profiling(mm_ctx* c, int32_t enable) {
  if (!c) return MM_EINVAL;
  c->adj_clean = false;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  unsigned long long ctr[C_N];
  HIP_OK(c, hipMemcpy(ctr, c->B.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  c->profiling = enable != 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  c->prof_u0 = ctr[C_UPDB0];
  c->prof_u1 = ctr[C_UPDB1];
  return MM_OK;
}

extern "C" mm_status mm_get_profile(mm_ctx* c, mm_profile* out) {
  if (!c || !out) return MM_EINVAL;
  c->adj_clean = false;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  unsigned long long ctr[C_N];
  HIP_OK(c, hipMemcpy(ctr, c->B.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
  double w = 8.0 * (c->P.dim + 2);
  double u0 = (double)(ctr[C_UPDB0] - c->prof_u0), u1 = (double)(ctr[C_UPDB1] - c->prof_u1);
  out->bulk_ms = c->prof_ms;
  out->bulk_launches = c->prof_launches;
  out->bulk_updates = (int64_t)(u0 + u1);
  out->bulk_bytes = u0 * 2.0 * w + u1 * 3.0 * w;
  return MM_OK;
}

// Multiresolution analysis (Sec. 2.4) of the current 2D state
__global__ void __launch_bounds__(256) k_mr_flags_u8(const uint32_t* a, uint8_t* out, long n) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = a[q] ? 1 : 0;
}
extern "C" mm_status mm_mr_analyse(mm_ctx* c, const mm_mr_params* p, int32_t* leaf_level,
                                   uint8_t* flags, mm_mr_result* res, int32_t ptr_kind) {
  if (!c || !p || !leaf_level || !res) return MM_EINVAL;
  c->adj_clean = false;
  if (!c->ready) return fail(c, MM_ESTATE, "mm_mr_analyse before mm_init_state");
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return fail(c, MM_EINVAL, "bad ptr_kind");
  const Params& P = c->P;
  int bs = p->block, L = p->levels;
  if (P.dim != 2) return fail(c, MM_EINVAL, "multiresolution analysis is built for 2D");
  if (bs < 2 || L < 1 || L > MR_MAXL || !(p->eps > 0.0) || std::isnan(p->band))
    return fail(c, MM_EINVAL, "block >= 2, 1 <= levels <= MM_MR_MAXL, eps > 0 required");
  long unit = (long)bs << L;
  if (P.nx % unit || P.ny % unit)
    return fail(c, MM_EINVAL, "nx and ny must be multiples of block * 2^levels");
  MrLevels V;
  memset(&V, 0, sizeof(V));
  V.L = L;
  long nflag = 0;
  size_t ncell[MR_MAXL + 1], cell_off[MR_MAXL + 1], ncells = 0;
  for (int l = 0; l <= L; l++) {
    V.nbx[l] = P.nx / (bs << (L - l));
    V.nby[l] = P.ny / (bs << (L - l));
    V.off[l] = nflag;
    nflag += (long)V.nbx[l] * V.nby[l];
    ncell[l] = ((size_t)P.nx >> (L - l)) * ((size_t)P.ny >> (L - l));
    cell_off[l] = ncells;
    ncells += ncell[l];
  }
  // layout: two pyramids of doubles, four flag arrays, the maxima, counts
  size_t b_u = 2 * ncells * sizeof(double), b_f = 4 * (size_t)nflag * sizeof(uint32_t);
  dim3 gf((P.nx + MR_TILE - 1) / MR_TILE, (P.ny + MR_TILE - 1) / MR_TILE);
  long nwg = (long)gf.x * gf.y;
  size_t need = b_u + b_f + 2 * sizeof(unsigned long long) +
                2 * (MR_MAXL + 1) * sizeof(unsigned long long) + 2 * nwg * sizeof(double) + 256;
  if (c->mr_cap < need) {
    if (c->mr_buf) (void)hipFree(c->mr_buf);
    c->mr_buf = nullptr;
    c->mr_cap = 0;
    if (hipMalloc(&c->mr_buf, need) != hipSuccess) return fail(c, MM_ENOMEM, "multiresolution buffers");
    c->mr_cap = need;
  }
  double* u0 = (double*)c->mr_buf;
  double* u1 = u0 + ncells;
  uint32_t* detail = (uint32_t*)(u1 + ncells);
  uint32_t* iface = detail + nflag;
  uint32_t* refine = iface + nflag;
  uint32_t* exist = refine + nflag;
  // four arrays of nflag words: 16 nflag bytes, so the maxima stay aligned
  unsigned long long* smax = (unsigned long long*)(exist + nflag);
  unsigned long long* counts = smax + 2;
  double* part = (double*)(counts + 2 * (MR_MAXL + 1));
  // clear flags and maxima (a fill kernel, not a memset node)
  Copies z;
  z.fill0(detail, 4 * (size_t)nflag * sizeof(uint32_t) + 2 * sizeof(unsigned long long));
  z.run(c);
  LAUNCH(k_mr_fields, gf, dim3(256), P, c->B, u0 + cell_off[L], u1 + cell_off[L],
         iface + V.off[L], bs, p->band, part);
  LAUNCH(k_mr_max, dim3(1), dim3(1024), part, nwg, smax);
  for (int l = L - 1; l >= 0; l--)
    LAUNCH(k_mr_project, lin_grid((long)ncell[l]), dim3(256), u0 + cell_off[l + 1],
           u1 + cell_off[l + 1], u0 + cell_off[l], u1 + cell_off[l], (int)(P.nx >> (L - l)),
           (int)(P.ny >> (L - l)));
  for (int l = 0; l < L; l++) {
    double e = std::ldexp(1.0, 2 * (l + 1 - L)) * p->eps;
    int nxf = (int)(P.nx >> (L - l - 1)), nyf = (int)(P.ny >> (L - l - 1));
    LAUNCH(k_mr_detail, dim3((nxf + MR_TILE - 1) / MR_TILE, (nyf + MR_TILE - 1) / MR_TILE),
           dim3(256), u0 + cell_off[l],
           u1 + cell_off[l], u0 + cell_off[l + 1], u1 + cell_off[l + 1],
           (int)(P.nx >> (L - l)), (int)(P.ny >> (L - l)), bs, e, smax, detail + V.off[l]);
  }
  int32_t* dleaf = leaf_level;
  uint8_t* dflags = flags;
  long nleaf = (long)V.nbx[L] * V.nby[L];
  long nfl = (V.off[L] /* detail of levels < L */) + nflag /* identifiers */;
  if (ptr_kind == MM_HOST) {
    size_t need_in = nleaf * sizeof(int32_t) + (flags ? nfl : 0) + 64;
    if (c->d_in_bytes < need_in) {
      if (c->d_in) (void)hipFree(c->d_in);
      c->d_in = nullptr;
      c->d_in_bytes = 0;
      if (hipMalloc(&c->d_in, need_in) != hipSuccess) return fail(c, MM_ENOMEM, "staging buffer");
      c->d_in_bytes = need_in;
    }
    dleaf = (int32_t*)c->d_in;
    dflags = flags ? (uint8_t*)(dleaf + nleaf) : nullptr;
  }
  LAUNCH(k_mr_tree, dim3(1), dim3(1024), V, detail, iface, refine, exist, dleaf, counts);
  if (dflags) {
    LAUNCH(k_mr_flags_u8, lin_grid(V.off[L]), dim3(256), detail, dflags, V.off[L]);
    LAUNCH(k_mr_flags_u8, lin_grid(nflag), dim3(256), iface, dflags + V.off[L], nflag);
  }
  HIP_OK(c, hipGetLastError());
  unsigned long long hc[2 * (MR_MAXL + 1) + 2];
  HIP_OK(c, hipMemcpyAsync(hc, smax, (2 + 2 * (L + 1)) * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
  if (ptr_kind == MM_HOST) {
    HIP_OK(c, hipMemcpyAsync(leaf_level, dleaf, nleaf * sizeof(int32_t), hipMemcpyDeviceToHost,
                             c->stream));
    if (flags)
      HIP_OK(c, hipMemcpyAsync(flags, dflags, nfl, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  memset(res, 0, sizeof(*res));
  double cells = 0.0;
  for (int l = 0; l <= L; l++) {
    res->exist[l] = (int64_t)hc[2 + 2 * l];
    res->leaf[l] = (int64_t)hc[2 + 2 * l + 1];
    cells += (double)res->leaf[l] * bs * bs;
  }
  res->compression = cells / ((double)P.nx * P.ny);
  memcpy(&res->scale[0], &hc[0], sizeof(double));
  memcpy(&res->scale[1], &hc[1], sizeof(double));
  return MM_OK;
}

#include "mmfv_batch.h"

#include "mmfv_adjoint_host.h"

// Steps with the tape kept: a checkpoint of the state every K steps and the
// step size of every step.  A new tape starts when none is open, when K
// changes, or once reverse steps have been taken.
// the counters of moves between materials (sum), after the queued work
static mm_status moves_count(mm_ctx* c, unsigned long long* out) {
  unsigned long long v[3];
  static_assert(C_RELABEL == C_ABSORB + 1 && C_ODDBALL == C_ABSORB + 2, "adjacent counters");
  HIP_OK(c, hipMemcpyAsync(v, c->B.ctr + C_ABSORB, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  *out = v[0] + v[1] + v[2];
  return MM_OK;
}

static mm_status step_record(mm_ctx* c, int32_t n_steps, int32_t K, double* t_out) {
  if (c->tape_K != K || c->tape_rev != c->tape_n) {
    c->tape_K = K;
    c->tape_n = c->tape_rev = 0;
    c->seg_n0 = -1;
    c->tape_moved = false;
  }
  unsigned long long moves0 = 0, moves1 = 0;
  mm_status mst = moves_count(c, &moves0);
  if (mst != MM_OK) return mst;
  size_t need = (size_t)(c->tape_n + n_steps) * sizeof(double);
  if (need > c->tape_dt_cap) {
    double* nd = nullptr;
    size_t cap = need * 2;
    HIP_OK(c, hipMalloc((void**)&nd, cap));
    if (c->tape_dt && c->tape_n)
      HIP_OK(c, hipMemcpyAsync(nd, c->tape_dt, c->tape_n * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (c->tape_dt) (void)hipFree(c->tape_dt);
    c->tape_dt = nd;
    c->tape_dt_cap = cap;
  }
  SnapLayout L = snap_layout(c->P);
  for (int n = 0; n < n_steps; n++) {
    if (c->tape_n % K == 0) {
      size_t q = (size_t)(c->tape_n / K);
      if (q >= c->ckpt.size()) {
        char* p = nullptr;
        HIP_OK(c, hipMalloc((void**)&p, L.bytes));
        c->ckpt.push_back(p);
      }
      Copies cp;
      snap_save(c, c->ckpt[q], 0, cp);
      cp.run(c);
    }
    mm_status st = launch_steps(c, 1);
    if (st != MM_OK) return st;
    cpy(c, c->tape_dt + c->tape_n, c->B.scal + S_DT, sizeof(double));
    c->tape_n++;
    c->tape_rev = c->tape_n;
  }
  c->seg_n0 = -1;
  mm_status st = finish_steps(c, t_out);
  if (st != MM_OK) return st;
  mst = moves_count(c, &moves1);
  if (mst != MM_OK) return mst;
  if (moves1 != moves0) c->tape_moved = true;
  return MM_OK;
}

// Guard of plain steps: the state a call starts from (snapshot with counters,
// scalars and sums); on a failure it is restored and the completed steps are
// replayed (the steps are deterministic, so the replay reproduces them bit for
// bit), leaving the state after the last completed step.
static mm_status guard_save(mm_ctx* c) {
  SnapLayout L = snap_layout(c->P);
  HIP_OK(c, grow(c, &c->guard_snap, &c->guard_cap, L.bytes));
  if (!c->guard_ctr) {
    HIP_OK(c, hipMalloc((void**)&c->guard_ctr, C_N * sizeof(unsigned long long)));
    HIP_OK(c, hipMalloc((void**)&c->guard_scal, 8 * sizeof(double)));
    HIP_OK(c, hipMalloc((void**)&c->guard_cons, CONS_N * sizeof(double)));
  }
  Copies cp;
  snap_save(c, c->guard_snap, 0, cp);
  cp.add(c->guard_ctr, c->B.ctr, C_N * sizeof(unsigned long long));
  cp.add(c->guard_scal, c->B.scal, 8 * sizeof(double));
  cp.add(c->guard_cons, c->B.cons, CONS_N * sizeof(double));
  cp.run(c);
  HIP_OK(c, hipGetLastError());
  return MM_OK;
}

static mm_status guard_rollback(mm_ctx* c, int64_t steps0, int64_t done) {
  // counters as at the start of the call, but the mixing stamp (it only
  // grows) and the tile count (the tile list is rebuilt)
  static_assert(C_STAMP + 1 == C_NTILES, "counters restored in two ranges");
  Copies rs;
  rs.add(c->B.scal, c->guard_scal, 8 * sizeof(double));
  rs.add(c->B.cons, c->guard_cons, CONS_N * sizeof(double));
  rs.add(c->B.ctr, c->guard_ctr, C_STAMP * sizeof(unsigned long long));
  rs.add(c->B.ctr + C_NTILES + 1, c->guard_ctr + C_NTILES + 1,
         (C_N - C_NTILES - 1) * sizeof(unsigned long long));
  if (c->D == 2) snap_load<2>(c, c->guard_snap, 0, &rs, true);
  else snap_load<1>(c, c->guard_snap, 0, &rs, true);
  c->steps = steps0;
  mm_status st = launch_steps(c, (int32_t)done);
  if (st != MM_OK) return st;
  unsigned long long err = 0;
  HIP_OK(c, hipMemcpyAsync(&err, c->B.ctr + C_ERR, sizeof(err), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (err != NO_ERR) {
    c->ready = false;
    return fail(c, MM_ENONPHYS, "the replay of the completed steps failed");
  }
  return MM_OK;
}
