// Host side of the batched C ABI (mm_batch_*): many independent 1D
// instances of uneven size advanced by one persistent launch.  Included once,
// at the end of mmfv_lib.hip.
#pragma once
#include <map>

struct mm_batch {
  int n = 0, M = 0, rk = 3;
  std::vector<mm_config> cfg;
  std::vector<Params> hP;
  std::vector<Bufs> hB;
  std::vector<int64_t> off;  // cell offsets of the instances, n + 1 entries
  Params* dP = nullptr;
  Bufs* dB = nullptr;
  int64_t* doff = nullptr;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  char* backup = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int threads = 0;  // workgroup size; 0 = choose by measurement
  bool ready = false;
  int64_t steps = 0;
  std::string err;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_objs;
  void* d_in = nullptr;
  size_t d_in_bytes = 0;
  unsigned long long* d_err = nullptr;
  float tune_ms[5] = {0, 0, 0, 0, 0};
};

static mm_status bfail(mm_batch* b, mm_status s, const std::string& msg) {
  if (b) b->err = msg;
  else g_create_err = msg;
  return s;
}
#define BHIP_OK(b, call)                                                    \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return bfail(b, MM_EDEVICE, std::string(#call) + ": " +               \
                                      hipGetErrorString(e_));               \
  } while (0)

// Assign the buffers of one instance from base (or only count bytes when
// base is NULL); every buffer starts on a 256-byte boundary.
static size_t layout_bufs(const Params& P, Bufs& B, char* base) {
  size_t at = 0, nc = P.NC, M = P.M, nv = P.dim + 2;
  auto take = [&](auto*& p, size_t count) {
    using T = std::remove_reference_t<decltype(*p)>;
    at = (at + 255) & ~(size_t)255;
    p = base ? (T*)(base + at) : nullptr;
    at += count * sizeof(T);
  };
  for (int b = 0; b < 3; b++) {
    take(B.Q[b], M * nv * nc);
    take(B.occ[b], nc);
  }
  take(B.phi, nc); take(B.ptmp, nc); take(B.phin, nc);
  take(B.chi, nc); take(B.ctmp, nc); take(B.chin, nc);
  take(B.al, M * nc); take(B.ax, M * nc); take(B.ay, M * nc);
  take(B.cx, M * nc); take(B.cy, M * nc);
  take(B.W, M * 4 * nc); take(B.Wit, M * nc);
  take(B.cut, nc); take(B.xs, nc); take(B.dcut, nc); take(B.dls, nc);
  take(B.rowc, nc); take(B.rowl, nc); take(B.tdc, nc); take(B.tdl, nc);
  take(B.nrow, nc); take(B.near4, nc);
  take(B.bulk, nc);
  take(B.X, M * 4 * nc);
  take(B.vx, nc); take(B.vy, nc); take(B.vit, nc);
  take(B.mixM, M * 3 * 4 * nc); take(B.mixT, M * 3 * nc);
  take(B.srcStamp, M * nc); take(B.tgtStamp, M * nc);
  take(B.tiles, 1);
  take(B.blist, 1);
  B.glist = nullptr;  // the batched kernel sweeps cells, not a queue
  take(B.scal, 8); take(B.ctr, C_N);
  take(B.vfc, nc);
  take(B.cons, CONS_N);
  B.cpart = nullptr;  // each instance reduces within its own workgroup
  return (at + 255) & ~(size_t)255;
}

__global__ void k_batch_ctr_init(const Bufs* Ba, int n) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int c = 0; c < C_N; c++) Ba[q].ctr[c] = 0;
  Ba[q].ctr[C_ERR] = NO_ERR;
  Ba[q].ctr[C_STAMP] = 1;  // stamp arrays start zeroed
  for (int c = 0; c < 8; c++) Ba[q].scal[c] = 0.0;
  for (int c = 0; c < CONS_N; c++) Ba[q].cons[c] = 0.0;
}
__global__ void k_batch_err(const Bufs* Ba, int n, unsigned long long* out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = Ba[q].ctr[C_ERR];
}
__global__ void k_batch_diag(const Bufs* Ba, int n, unsigned long long* ctr, double* scal,
                             double* cons) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int c = 0; c < C_N; c++) ctr[(size_t)q * C_N + c] = Ba[q].ctr[c];
  for (int c = 0; c < 8; c++) scal[(size_t)q * 8 + c] = Ba[q].scal[c];
  for (int c = 0; c < CONS_N; c++) cons[(size_t)q * CONS_N + c] = Ba[q].cons[c];
}

static void batch_free(mm_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : b->graph_objs) (void)hipGraphDestroy(g);
  b->graphs.clear();
  b->graph_objs.clear();
  void* ps[] = {b->dP, b->dB, b->doff, b->pool, b->backup, b->d_in, b->d_err};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

extern "C" mm_status mm_batch_create(const mm_config* cfgs, int32_t n_inst, void* hip_stream,
                                     mm_batch** out) {
  if (!cfgs || !out || n_inst < 1) return bfail(nullptr, MM_EINVAL, "bad arguments");
  std::string why;
  for (int q = 0; q < n_inst; q++) {
    if (!valid_config(&cfgs[q], why)) return bfail(nullptr, MM_EINVAL, why);
    if (cfgs[q].dim != 1) return bfail(nullptr, MM_EINVAL, "batched instances must be 1D");
    if (cfgs[q].n_mat != cfgs[0].n_mat || cfgs[q].rk_order != cfgs[0].rk_order)
      return bfail(nullptr, MM_EINVAL, "instances must share n_mat and rk_order");
  }
  mm_batch* b = new mm_batch();
  b->n = n_inst;
  b->M = cfgs[0].n_mat;
  b->rk = cfgs[0].rk_order;
  b->cfg.assign(cfgs, cfgs + n_inst);
  b->hP.resize(n_inst);
  b->hB.resize(n_inst);
  b->off.assign(n_inst + 1, 0);
  std::vector<size_t> start(n_inst);
  size_t total = 0;
  for (int q = 0; q < n_inst; q++) {
    b->hP[q] = make_params(&cfgs[q]);
    start[q] = total;
    total += layout_bufs(b->hP[q], b->hB[q], nullptr);
    b->off[q + 1] = b->off[q] + cfgs[q].nx;
  }
  b->pool_bytes = total;
  hipError_t e = hipMalloc((void**)&b->pool, total);
  if (e == hipSuccess) e = hipMemset(b->pool, 0, total);
  if (e == hipSuccess) e = hipMalloc((void**)&b->dP, sizeof(Params) * n_inst);
  if (e == hipSuccess) e = hipMalloc((void**)&b->dB, sizeof(Bufs) * n_inst);
  if (e == hipSuccess) e = hipMalloc((void**)&b->doff, sizeof(int64_t) * (n_inst + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_err, sizeof(unsigned long long) * n_inst);
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return bfail(nullptr, e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EDEVICE, "allocation");
  }
  for (int q = 0; q < n_inst; q++) layout_bufs(b->hP[q], b->hB[q], b->pool + start[q]);
  e = hipMemcpy(b->dP, b->hP.data(), sizeof(Params) * n_inst, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->dB, b->hB.data(), sizeof(Bufs) * n_inst, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->doff, b->off.data(), sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else if (e == hipSuccess) {
    e = hipStreamCreate(&b->stream);  // graph capture needs a non-null stream
    b->own_stream = true;
  }
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return bfail(nullptr, MM_EDEVICE, "setup");
  }
  *out = b;
  return MM_OK;
}

extern "C" mm_status mm_batch_destroy(mm_batch* b) {
  if (!b) return MM_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  delete b;
  return MM_OK;
}

extern "C" const char* mm_batch_last_error(const mm_batch* b) {
  return b ? b->err.c_str() : g_create_err.c_str();
}

static int batch_threads_for(const mm_batch* b) { return b->threads > 0 ? b->threads : 256; }

extern "C" mm_status mm_batch_init_state(mm_batch* b, const double* phi, const int32_t* chi,
                                         const double* W, int32_t ptr_kind) {
  if (!b) return MM_EINVAL;
  if (!phi || !chi || !W) return bfail(b, MM_EINVAL, "NULL input array");
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return bfail(b, MM_EINVAL, "bad ptr_kind");
  int64_t ncell = b->off[b->n];
  size_t nW = (size_t)b->M * 3 * ncell;
  const double *dphi = phi, *dW = W;
  const int32_t* dchi = chi;
  if (ptr_kind == MM_HOST) {
    for (int64_t q = 0; q < ncell; q++)
      if (chi[q] < 0 || chi[q] >= b->M || !(phi[q] >= 0.0))
        return bfail(b, MM_EINVAL, "chi out of range or phi negative");
    size_t need = (ncell + nW) * sizeof(double) + ncell * sizeof(int32_t);
    if (b->d_in_bytes < need) {
      if (b->d_in) (void)hipFree(b->d_in);
      b->d_in = nullptr;
      b->d_in_bytes = 0;
      if (hipMalloc(&b->d_in, need) != hipSuccess) return bfail(b, MM_ENOMEM, "staging");
      b->d_in_bytes = need;
    }
    double* p0 = (double*)b->d_in;
    double* w0 = p0 + ncell;
    int32_t* c0 = (int32_t*)(w0 + nW);
    BHIP_OK(b, hipMemcpyAsync(p0, phi, ncell * sizeof(double), hipMemcpyHostToDevice, b->stream));
    BHIP_OK(b, hipMemcpyAsync(w0, W, nW * sizeof(double), hipMemcpyHostToDevice, b->stream));
    BHIP_OK(b, hipMemcpyAsync(c0, chi, ncell * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    dphi = p0;
    dW = w0;
    dchi = c0;
  }
  BHIP_OK(b, hipMemsetAsync(b->pool, 0, b->pool_bytes, b->stream));
  hipLaunchKernelGGL(k_batch_ctr_init, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB,
                     b->n);
  hipLaunchKernelGGL(k_batch1d_init, dim3(b->n), dim3(batch_threads_for(b)), 0, b->stream, b->dP,
                     b->dB, dphi, dchi, dW, (const int64_t*)b->doff);
  BHIP_OK(b, hipGetLastError());
  hipLaunchKernelGGL(k_batch_err, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB, b->n,
                     b->d_err);
  std::vector<unsigned long long> err(b->n);
  BHIP_OK(b, hipMemcpyAsync(err.data(), b->d_err, sizeof(unsigned long long) * b->n,
                            hipMemcpyDeviceToHost, b->stream));
  BHIP_OK(b, hipStreamSynchronize(b->stream));
  b->steps = 0;
  b->ready = true;
  for (int q = 0; q < b->n; q++)
    if (err[q] != NO_ERR) {
      b->ready = false;
      return bfail(b, MM_ENONPHYS, "instance " + std::to_string(q) + ": non-physical cell " +
                                       std::to_string(err[q]));
    }
  return MM_OK;
}

static void batch_launch_direct(mm_batch* b, int n_steps, int threads) {
  auto kern = threads <= 256 ? k_batch1d<256> : (threads <= 512 ? k_batch1d<512> : k_batch1d<1024>);
  hipLaunchKernelGGL(kern, dim3(b->n), dim3(threads), 0, b->stream,
                     (const Params*)b->dP, (const Bufs*)b->dB, n_steps, b->rk);
}

// one persistent launch, replayed from a HIP graph captured per (steps,
// workgroup size); falls back to a direct launch if capture is unavailable
static mm_status batch_launch(mm_batch* b, int n_steps, int threads) {
  auto key = std::make_pair(n_steps, threads);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool ok = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      batch_launch_direct(b, n_steps, threads);
      ok = hipStreamEndCapture(b->stream, &g) == hipSuccess && g != nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      batch_launch_direct(b, n_steps, threads);
      BHIP_OK(b, hipGetLastError());
      return MM_OK;
    }
    b->graph_objs.push_back(g);
    it = b->graphs.emplace(key, x).first;
  }
  BHIP_OK(b, hipGraphLaunch(it->second, b->stream));
  return MM_OK;
}

// Choose the workgroup size by timing a few steps with each candidate on a
// snapshot of the state; the snapshot is restored afterwards, so tuning does
// not change any result.
static mm_status batch_autotune(mm_batch* b, int trial_steps) {
  static const int cand[5] = {64, 128, 256, 512, 1024};
  if (!b->backup) BHIP_OK(b, hipMalloc((void**)&b->backup, b->pool_bytes));
  BHIP_OK(b, hipMemcpyAsync(b->backup, b->pool, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream));
  hipEvent_t e0, e1;
  BHIP_OK(b, hipEventCreate(&e0));
  BHIP_OK(b, hipEventCreate(&e1));
  float best = 1e30f;
  int bestT = 256;
  for (int c = 0; c < 5; c++) {
    batch_launch_direct(b, 1, cand[c]);  // warm-up of this shape
    BHIP_OK(b, hipEventRecord(e0, b->stream));
    batch_launch_direct(b, trial_steps, cand[c]);
    BHIP_OK(b, hipEventRecord(e1, b->stream));
    BHIP_OK(b, hipEventSynchronize(e1));
    float ms = 0.f;
    BHIP_OK(b, hipEventElapsedTime(&ms, e0, e1));
    b->tune_ms[c] = ms;
    if (ms < best) {
      best = ms;
      bestT = cand[c];
    }
    BHIP_OK(b, hipMemcpyAsync(b->pool, b->backup, b->pool_bytes, hipMemcpyDeviceToDevice,
                              b->stream));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  BHIP_OK(b, hipStreamSynchronize(b->stream));
  b->threads = bestT;
  return MM_OK;
}

extern "C" mm_status mm_batch_set_threads(mm_batch* b, int32_t threads) {
  if (!b) return MM_EINVAL;
  if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512 &&
      threads != 1024)
    return bfail(b, MM_EINVAL, "threads must be 0 (tune) or 64..1024, a power of two");
  b->threads = threads;
  return MM_OK;
}

extern "C" mm_status mm_batch_get_threads(mm_batch* b, int32_t* threads, float* tune_ms) {
  if (!b || !threads) return MM_EINVAL;
  *threads = b->threads;
  if (tune_ms)
    for (int c = 0; c < 5; c++) tune_ms[c] = b->tune_ms[c];
  return MM_OK;
}

extern "C" mm_status mm_batch_step(mm_batch* b, int32_t n_steps) {
  if (!b) return MM_EINVAL;
  if (!b->ready) return bfail(b, MM_ESTATE, "mm_batch_step before mm_batch_init_state");
  if (n_steps < 0) return bfail(b, MM_EINVAL, "n_steps < 0");
  if (n_steps == 0) return MM_OK;
  if (b->threads == 0) {
    mm_status st = batch_autotune(b, 3);
    if (st != MM_OK) return st;
  }
  mm_status st = batch_launch(b, n_steps, b->threads);
  if (st != MM_OK) return st;
  hipLaunchKernelGGL(k_batch_err, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB, b->n,
                     b->d_err);
  std::vector<unsigned long long> err(b->n);
  BHIP_OK(b, hipMemcpyAsync(err.data(), b->d_err, sizeof(unsigned long long) * b->n,
                            hipMemcpyDeviceToHost, b->stream));
  BHIP_OK(b, hipStreamSynchronize(b->stream));
  b->steps += n_steps;
  for (int q = 0; q < b->n; q++)
    if (err[q] != NO_ERR) {
      b->ready = false;
      return bfail(b, MM_ENONPHYS, "instance " + std::to_string(q) + ": non-physical cell " +
                                       std::to_string(err[q]));
    }
  return MM_OK;
}

extern "C" mm_status mm_batch_get_conserved(mm_batch* b, double* Q, double* alpha, double* phi,
                                            int32_t* chi, int32_t ptr_kind) {
  if (!b) return MM_EINVAL;
  if (!Q) return bfail(b, MM_EINVAL, "Q must not be NULL");
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return bfail(b, MM_EINVAL, "bad ptr_kind");
  int64_t ncell = b->off[b->n];
  size_t nQ = (size_t)b->M * 3 * ncell, nA = (size_t)b->M * ncell;
  int T = batch_threads_for(b);
  if (ptr_kind == MM_DEVICE) {
    hipLaunchKernelGGL(k_batch1d_pack, dim3(b->n), dim3(T), 0, b->stream, b->dP, b->dB, Q, alpha,
                       phi, chi, (const int64_t*)b->doff);
    BHIP_OK(b, hipGetLastError());
    return MM_OK;
  }
  size_t need = (nQ + nA + ncell) * sizeof(double) + ncell * sizeof(int32_t);
  if (b->d_in_bytes < need) {
    if (b->d_in) (void)hipFree(b->d_in);
    b->d_in = nullptr;
    b->d_in_bytes = 0;
    if (hipMalloc(&b->d_in, need) != hipSuccess) return bfail(b, MM_ENOMEM, "staging");
    b->d_in_bytes = need;
  }
  double* q0 = (double*)b->d_in;
  double* a0 = q0 + nQ;
  double* p0 = a0 + nA;
  int32_t* c0 = (int32_t*)(p0 + ncell);
  hipLaunchKernelGGL(k_batch1d_pack, dim3(b->n), dim3(T), 0, b->stream, b->dP, b->dB, q0, a0, p0,
                     c0, (const int64_t*)b->doff);
  BHIP_OK(b, hipGetLastError());
  BHIP_OK(b, hipMemcpyAsync(Q, q0, nQ * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if (alpha)
    BHIP_OK(b, hipMemcpyAsync(alpha, a0, nA * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if (phi)
    BHIP_OK(b, hipMemcpyAsync(phi, p0, ncell * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  if (chi)
    BHIP_OK(b, hipMemcpyAsync(chi, c0, ncell * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
  BHIP_OK(b, hipStreamSynchronize(b->stream));
  return MM_OK;
}

extern "C" mm_status mm_batch_get_diagnostics(mm_batch* b, mm_diag* out) {
  if (!b || !out) return MM_EINVAL;
  unsigned long long* dctr = nullptr;
  double* dscal = nullptr;
  double* dcons = nullptr;
  hipError_t e = hipMalloc((void**)&dctr, sizeof(unsigned long long) * C_N * b->n);
  if (e == hipSuccess) e = hipMalloc((void**)&dscal, sizeof(double) * 8 * b->n);
  if (e == hipSuccess) e = hipMalloc((void**)&dcons, sizeof(double) * CONS_N * b->n);
  std::vector<unsigned long long> ctr((size_t)C_N * b->n);
  std::vector<double> scal((size_t)8 * b->n), cons((size_t)CONS_N * b->n);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_batch1d_qsum, dim3(b->n), dim3(256), 0, b->stream, b->dP, b->dB);
    hipLaunchKernelGGL(k_batch_diag, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB,
                       b->n, dctr, dscal, dcons);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctr.data(), dctr, ctr.size() * sizeof(ctr[0]), hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(scal.data(), dscal, scal.size() * sizeof(double), hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cons.data(), dcons, cons.size() * sizeof(double), hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (dctr) (void)hipFree(dctr);
  if (dscal) (void)hipFree(dscal);
  if (dcons) (void)hipFree(dcons);
  if (e != hipSuccess) return bfail(b, MM_EDEVICE, hipGetErrorString(e));
  for (int q = 0; q < b->n; q++) {
    const unsigned long long* c = &ctr[(size_t)q * C_N];
    const double* s = &scal[(size_t)q * 8];
    mm_diag& d = out[q];
    d.t = s[S_T];
    d.dt = s[S_DT];
    d.steps = b->steps;
    d.n_posfix = (int64_t)c[C_POSFIX];
    d.n_fluxskip = (int64_t)c[C_FLUXSKIP];
    d.n_ifskip = (int64_t)c[C_IFSKIP];
    d.n_stranded = (int64_t)c[C_STRANDED];
    d.n_mixsrc = (int64_t)c[C_MIXSRC];
    d.n_updates = (int64_t)c[C_UPD];
    d.err_cell = c[C_ERR] == NO_ERR ? -1 : (int64_t)c[C_ERR];
    d.n_band = d.n_ghost = d.n_tiles = 0;
    cons_to_diag(&cons[(size_t)q * CONS_N], b->M, &d);
  }
  return MM_OK;
}
