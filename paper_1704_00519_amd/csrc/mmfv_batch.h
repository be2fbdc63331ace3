// Host side of the batched C ABI (mm_batch_*): many independent 1D
// instances of uneven size advanced by one persistent launch.  Included once,
// at the end of mmfv_lib.hip.
#pragma once
#include <algorithm>
#include <map>
#include <mutex>

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
  take(B.strStamp, M * nc); take(B.abMark, nc); take(B.rlStamp, nc);
  take(B.rlTo, nc); take(B.ssTo, nc); take(B.abList, nc); take(B.ssList, nc);
  take(B.ssPhi, nc);
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
  Ba[q].ctr[C_ERRSTEP] = NO_ERR;
  Ba[q].ctr[C_STAMP] = 1;  // stamp arrays start zeroed
  for (int c = 0; c < 8; c++) Ba[q].scal[c] = 0.0;
  for (int c = 0; c < CONS_N; c++) Ba[q].cons[c] = 0.0;
}
__global__ void k_batch_err(const Bufs* Ba, int n, unsigned long long* out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = Ba[q].ctr[C_ERR];
}
__global__ void k_batch_badin(const Bufs* Ba, int n, unsigned long long* out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = Ba[q].ctr[C_BADIN];
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
  std::vector<unsigned long long> err(b->n);
  if (ptr_kind == MM_DEVICE) {
    hipLaunchKernelGGL(k_batch_badin, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB,
                       b->n, b->d_err);
    BHIP_OK(b, hipMemcpyAsync(err.data(), b->d_err, sizeof(unsigned long long) * b->n,
                              hipMemcpyDeviceToHost, b->stream));
    BHIP_OK(b, hipStreamSynchronize(b->stream));
    for (int q = 0; q < b->n; q++)
      if (err[q] != 0) {
        b->ready = false;
        return bfail(b, MM_EINVAL, "instance " + std::to_string(q) +
                                       ": chi out of range or phi negative");
      }
  }
  hipLaunchKernelGGL(k_batch_err, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->dB, b->n,
                     b->d_err);
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
    d.n_absorb = (int64_t)c[C_ABSORB];
    d.n_relabel = (int64_t)c[C_RELABEL];
    d.n_oddball = (int64_t)c[C_ODDBALL];
    d.n_mixsrc = (int64_t)c[C_MIXSRC];
    d.n_updates = (int64_t)c[C_UPD];
    d.err_cell = c[C_ERR] == NO_ERR ? -1 : (int64_t)c[C_ERR];
    d.err_step = c[C_ERRSTEP] == NO_ERR ? -1 : (int64_t)c[C_ERRSTEP] + 1;
    d.n_band = d.n_ghost = d.n_tiles = 0;
    cons_to_diag(&cons[(size_t)q * CONS_N], b->M, &d);
  }
  return MM_OK;
}

// ---------------------------------------------------------------------------
// Batched run with no device allocation (mm_batch_run_noalloc)
// ---------------------------------------------------------------------------
// Every buffer of the run (instance parameters and buffer tables, offsets,
// error words and the instances' state and work buffers) lives in one
// file-scope device array.  Host code never passes the array's name to a
// kernel or copy: it uses the device address obtained once per device with
// hipGetSymbolAddress.  Calls on one GPU share the array, so calls that
// overlap on one GPU race.
static __device__ __align__(256) char scratch[MM_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

// device address of this device's scratch array (looked up once per device)
static hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return hipSuccess;
}

__global__ void __launch_bounds__(256) k_fill0(char* p, size_t bytes) {
  size_t words = bytes / 8;
  double* d = (double*)p;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
       w += (size_t)gridDim.x * blockDim.x)
    d[w] = 0.0;
}

// the lowest failing instance (n_inst if none) and its error word
__global__ void k_batch_first_err(const Bufs* Ba, int n, unsigned long long* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  out[0] = (unsigned long long)n;
  out[1] = NO_ERR;
  for (int q = 0; q < n; q++)
    if (Ba[q].ctr[C_ERR] != NO_ERR) {
      out[0] = (unsigned long long)q;
      out[1] = Ba[q].ctr[C_ERR];
      return;
    }
}

static size_t na_align(size_t n) { return (n + 255) & ~(size_t)255; }

extern "C" mm_status mm_batch_run_noalloc(const mm_config* cfgs, int32_t n_inst,
                                          void* hip_stream, const double* phi,
                                          const int32_t* chi, const double* W, int32_t n_steps,
                                          int32_t threads, double* Q, double* alpha,
                                          double* phi_out, int32_t* chi_out) {
  if (!cfgs || !phi || !chi || !W || !Q)
    return bfail(nullptr, MM_EINVAL, "noalloc: NULL argument");
  if (n_inst < 1 || n_inst > MM_NOALLOC_MAX_INST)
    return bfail(nullptr, MM_EINVAL, "noalloc: n_inst must be in [1, MM_NOALLOC_MAX_INST]");
  if (n_steps < 0) return bfail(nullptr, MM_EINVAL, "noalloc: n_steps < 0");
  if (threads == 0) threads = 256;
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return bfail(nullptr, MM_EINVAL, "noalloc: threads must be 0 or 64..1024, a power of two");
  std::string why;
  for (int q = 0; q < n_inst; q++) {
    if (!valid_config(&cfgs[q], why)) return bfail(nullptr, MM_EINVAL, "noalloc: " + why);
    if (cfgs[q].dim != 1) return bfail(nullptr, MM_EINVAL, "noalloc: instances must be 1D");
    if (cfgs[q].n_mat != cfgs[0].n_mat || cfgs[q].rk_order != cfgs[0].rk_order)
      return bfail(nullptr, MM_EINVAL, "noalloc: instances must share n_mat and rk_order");
  }
  // host-side tables in fixed storage (no allocation); one caller at a time
  // per thread
  static thread_local Params hP[MM_NOALLOC_MAX_INST];
  static thread_local Bufs hB[MM_NOALLOC_MAX_INST];
  static thread_local int64_t hoff[MM_NOALLOC_MAX_INST + 1];
  size_t at_P = 0, at_B = na_align(at_P + sizeof(Params) * n_inst);
  size_t at_off = na_align(at_B + sizeof(Bufs) * n_inst);
  size_t at_err = na_align(at_off + sizeof(int64_t) * (n_inst + 1));
  size_t at_pool = na_align(at_err + 2 * sizeof(unsigned long long));
  size_t pool = 0;
  hoff[0] = 0;
  for (int q = 0; q < n_inst; q++) {
    hP[q] = make_params(&cfgs[q]);
    pool += layout_bufs(hP[q], hB[q], nullptr);
    hoff[q + 1] = hoff[q] + cfgs[q].nx;
  }
  if (at_pool + pool > (size_t)MM_NOALLOC_BYTES)
    return bfail(nullptr, MM_EINVAL,
                 "noalloc: the instances need " + std::to_string(at_pool + pool) +
                     " bytes of work memory, more than MM_NOALLOC_BYTES");
  char* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess)
    return bfail(nullptr, MM_EDEVICE, std::string("noalloc: scratch address: ") +
                                          hipGetErrorString(e));
  size_t at = at_pool;
  for (int q = 0; q < n_inst; q++) at += layout_bufs(hP[q], hB[q], base + at);
  hipStream_t s = (hipStream_t)hip_stream;
  Params* dP = (Params*)(base + at_P);
  Bufs* dB = (Bufs*)(base + at_B);
  int64_t* doff = (int64_t*)(base + at_off);
  unsigned long long* derr = (unsigned long long*)(base + at_err);
#define NHIP(call)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return bfail(nullptr, MM_EDEVICE, std::string("noalloc: " #call ": ") +              \
                                            hipGetErrorString(e_));                        \
  } while (0)
  // the work buffers start at zero, as after mm_batch_init_state's clear
  unsigned gfill = (unsigned)std::min<size_t>(2048, (pool / 8 + 255) / 256 + 1);
  hipLaunchKernelGGL(k_fill0, dim3(gfill), dim3(256), 0, s, base + at_pool, pool);
  NHIP(hipMemcpyAsync(dP, hP, sizeof(Params) * n_inst, hipMemcpyHostToDevice, s));
  NHIP(hipMemcpyAsync(dB, hB, sizeof(Bufs) * n_inst, hipMemcpyHostToDevice, s));
  NHIP(hipMemcpyAsync(doff, hoff, sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_batch_ctr_init, dim3((n_inst + 255) / 256), dim3(256), 0, s, dB, n_inst);
  hipLaunchKernelGGL(k_batch1d_init, dim3(n_inst), dim3(threads), 0, s, (const Params*)dP,
                     (const Bufs*)dB, phi, chi, W, (const int64_t*)doff);
  if (n_steps > 0) {
    auto kern = threads <= 256 ? k_batch1d<256> : (threads <= 512 ? k_batch1d<512> : k_batch1d<1024>);
    hipLaunchKernelGGL(kern, dim3(n_inst), dim3(threads), 0, s, (const Params*)dP,
                       (const Bufs*)dB, n_steps, cfgs[0].rk_order);
  }
  hipLaunchKernelGGL(k_batch1d_pack, dim3(n_inst), dim3(threads), 0, s, (const Params*)dP,
                     (const Bufs*)dB, Q, alpha, phi_out, chi_out, (const int64_t*)doff);
  hipLaunchKernelGGL(k_batch_first_err, dim3(1), dim3(64), 0, s, (const Bufs*)dB, n_inst, derr);
  NHIP(hipGetLastError());
  unsigned long long herr[2] = {0, 0};
  NHIP(hipMemcpyAsync(herr, derr, sizeof(herr), hipMemcpyDeviceToHost, s));
  NHIP(hipStreamSynchronize(s));
#undef NHIP
  if (herr[0] != (unsigned long long)n_inst)
    return bfail(nullptr, MM_ENONPHYS, "noalloc: instance " + std::to_string(herr[0]) +
                                           ": non-physical cell " + std::to_string(herr[1]));
  return MM_OK;
}
