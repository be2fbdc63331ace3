// Host side of the adjoint entry points: the tape of recorded steps
// (checkpoints every K steps and the step sizes), recomputation of one
// segment with per-stage snapshots, and the reverse of one time step.
// Included once, at the end of mmfv_lib.hip.
#pragma once

// ---------------------------------------------------------------------------
// Snapshots of the state at the start of a stage: Q and occupancy of the
// stage's input buffer, the level set with its frame, the geometry and the
// record of the volume-fraction correction; after stage 0 of a step also
// the level-set velocity and the time-n level set.
// ---------------------------------------------------------------------------
struct SnapLayout {
  size_t q, phi, geo, occ, chi, vfc, cls, bytes;  // stage snapshot offsets
  size_t vx, vy, phin, chin, ext_bytes;      // step extras offsets
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static SnapLayout snap_layout(const Params& P) {
  SnapLayout L;
  size_t nc = P.NC, M = P.M, nv = P.dim + 2, at = 0;
  L.q = at; at = align256(at + M * nv * nc * 8);
  L.phi = at; at = align256(at + nc * 8);
  L.geo = at; at = align256(at + 5 * M * nc * 8);
  L.occ = at; at = align256(at + nc);
  L.chi = at; at = align256(at + nc);
  L.vfc = at; at = align256(at + nc * 2);
  L.cls = at; at = align256(at + 4 * nc);  // classification: cut, xs, dcut, dls
  L.bytes = at;
  at = 0;
  L.vx = at; at = align256(at + nc * 8);
  L.vy = at; at = align256(at + nc * 8);
  L.phin = at; at = align256(at + nc * 8);
  L.chin = at; at = align256(at + nc);
  L.ext_bytes = at;
  return L;
}

static void cpy(mm_ctx* c, void* dst, const void* src, size_t n) {
  (void)hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, c->stream);
}


static void geo_ptrs(mm_ctx* c, double* g[5]) {
  g[0] = c->B.al; g[1] = c->B.ax; g[2] = c->B.ay; g[3] = c->B.cx; g[4] = c->B.cy;
}

static void snap_save(mm_ctx* c, char* dst, int sidx, Copies& cp) {
  const Params& P = c->P;
  SnapLayout L = snap_layout(P);
  size_t nc = P.NC, M = P.M, nv = P.dim + 2;
  cp.add(dst + L.q, c->B.Q[sidx], M * nv * nc * 8);
  cp.add(dst + L.phi, c->B.phi, nc * 8);
  double* g[5];
  geo_ptrs(c, g);
  for (int q = 0; q < 5; q++) cp.add(dst + L.geo + q * M * nc * 8, g[q], M * nc * 8);
  cp.add(dst + L.occ, c->B.occ[sidx], nc);
  cp.add(dst + L.chi, c->B.chi, nc);
  cp.add(dst + L.vfc, c->B.vfc, nc * 2);
  uint8_t* cls[4] = {c->B.cut, c->B.xs, c->B.dcut, c->B.dls};
  for (int q = 0; q < 4; q++) cp.add(dst + L.cls + q * nc, cls[q], nc);
}

// restore a stage snapshot into buffer sidx (with optional extra copies in
// the same launch) with its classification (a function of the level set and
// the indicator, kept with the snapshot); the tile list is emptied and, with
// tiles, rebuilt
template <int D>
static void snap_load(mm_ctx* c, const char* src, int sidx, Copies* extra = nullptr,
                      bool tiles = true) {
  const Params& P = c->P;
  SnapLayout L = snap_layout(P);
  size_t nc = P.NC, M = P.M, nv = P.dim + 2;
  Copies own;
  Copies& cp = extra ? *extra : own;
  cp.add(c->B.Q[sidx], src + L.q, M * nv * nc * 8);
  cp.add(c->B.phi, src + L.phi, nc * 8);
  double* g[5];
  geo_ptrs(c, g);
  for (int q = 0; q < 5; q++) cp.add(g[q], src + L.geo + q * M * nc * 8, M * nc * 8);
  cp.add(c->B.occ[sidx], src + L.occ, nc);
  cp.add(c->B.chi, src + L.chi, nc);
  cp.add(c->B.vfc, src + L.vfc, nc * 2);
  uint8_t* cls[4] = {c->B.cut, c->B.xs, c->B.dcut, c->B.dls};
  for (int q = 0; q < 4; q++) cp.add(cls[q], src + L.cls + q * nc, nc);
  cp.fill0(&c->B.ctr[C_NTILES], sizeof(unsigned long long));
  // the quiet-block maps of the classification describe another state
  if (D == 2) {
    size_t ncb = (size_t)((P.nx + CX - 1) / CX) * ((P.ny + CY - 1) / CY);
    cp.fill0(c->B.cquiet[0], ncb);
    cp.fill0(c->B.cquiet[1], ncb);
  }
  cp.run(c);
  if (tiles) build_tiles<D>(c, sidx, 0);  // only forward kernels read the tile list
}

static void ext_save(mm_ctx* c, char* dst, Copies& cp) {
  SnapLayout L = snap_layout(c->P);
  size_t nc = c->P.NC;
  cp.add(dst + L.vx, c->B.vx, nc * 8);
  cp.add(dst + L.vy, c->B.vy, nc * 8);
  cp.add(dst + L.phin, c->B.phin, nc * 8);
  cp.add(dst + L.chin, c->B.chin, nc);
}
static void ext_add(mm_ctx* c, Copies& cp, const char* src) {
  SnapLayout L = snap_layout(c->P);
  size_t nc = c->P.NC;
  cp.add(c->B.vx, src + L.vx, nc * 8);
  cp.add(c->B.vy, src + L.vy, nc * 8);
  cp.add(c->B.phin, src + L.phin, nc * 8);
  cp.add(c->B.chin, src + L.chin, nc);
}

// Per stage, besides the snapshot: Q* (after the update, before mixing)
// with its occupancy, and the states the stage read: primitive states W and
// their validity marks, the ghost queue with its length, the velocity marks
struct StageExtra {
  size_t q, occ, W, Wit, glist, nghost, vit, bytes;
};
static StageExtra stage_extra(const Params& P) {
  StageExtra E;
  size_t nc = P.NC, M = P.M, at = 0;
  E.q = at; at = align256(at + M * (P.dim + 2) * nc * 8);
  E.occ = at; at = align256(at + nc);
  E.W = at; at = align256(at + M * 4 * nc * 8);
  E.Wit = at; at = align256(at + M * nc);
  E.glist = at; at = align256(at + M * nc * 4);
  E.nghost = at; at = align256(at + 8);
  E.vit = at; at = align256(at + nc);
  E.bytes = at;
  return E;
}
static size_t qstar_bytes(const Params& P) { return stage_extra(P).bytes; }
// segment buffer: per step, ns stage snapshots, ns stage extras, then the
// step extras
static size_t seg_step_bytes(const mm_ctx* c, int ns) {
  SnapLayout L = snap_layout(c->P);
  return ns * (L.bytes + qstar_bytes(c->P)) + L.ext_bytes;
}
static char* seg_stage(mm_ctx* c, int64_t rel, int s, int ns) {
  return c->seg + rel * seg_step_bytes(c, ns) + s * snap_layout(c->P).bytes;
}
static char* seg_qstar(mm_ctx* c, int64_t rel, int s, int ns) {
  return c->seg + rel * seg_step_bytes(c, ns) + ns * snap_layout(c->P).bytes +
         s * qstar_bytes(c->P);
}
static uint8_t* seg_qstar_occ(mm_ctx* c, int64_t rel, int s, int ns) {
  return (uint8_t*)(seg_qstar(c, rel, s, ns) + stage_extra(c->P).occ);
}
// the states read by stage s, kept / restored in the same layout
static void states_copies(mm_ctx* c, Copies& cp, char* blk, bool save) {
  StageExtra E = stage_extra(c->P);
  size_t nc = c->P.NC, M = c->P.M;
  void* dev[5] = {c->B.W, c->B.Wit, c->B.glist, &c->B.ctr[C_NGHOST], c->B.vit};
  size_t off[5] = {E.W, E.Wit, E.glist, E.nghost, E.vit};
  size_t n[5] = {M * 4 * nc * 8, M * nc, M * nc * 4, 8, nc};
  for (int q = 0; q < 5; q++) {
    if (save) cp.add(blk + off[q], dev[q], n[q]);
    else cp.add(dev[q], blk + off[q], n[q]);
  }
}
static char* seg_ext(mm_ctx* c, int64_t rel, int ns) {
  return c->seg + rel * seg_step_bytes(c, ns) +
         ns * (snap_layout(c->P).bytes + qstar_bytes(c->P));
}

static hipError_t grow(mm_ctx* c, char** p, size_t* cap, size_t need) {
  if (*cap >= need) return hipSuccess;
  if (*p) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(*p);
  }
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc((void**)p, need);
  if (e == hipSuccess) *cap = need;
  return e;
}

// recompute recorded steps [n0, n1) from the checkpoint at n0 and keep the
// stage snapshots of every step
template <int D>
static void load_segment(mm_ctx* c, int64_t n0, int64_t n1) {
  double b[3], cc[3], w[3];
  int ns = rk_coefs(c->cfg, b, cc, w);
  snap_load<D>(c, c->ckpt[n0 / c->tape_K], 0);
  // the copies ride on the stage's own launches: its input snapshot (and,
  // before a step, the recorded step size, which stage 0 takes over) on the
  // first, what it read (and after stage 0 the level-set velocity) on the
  // last; a list too long for that goes out on its own
  for (int64_t n = n0; n < n1; n++) {
    for (int s = 0; s < ns; s++) {
      int sidx = stage_src(s), didx = stage_dst(s, ns);
      Copies pre, post;
      if (s == 0) pre.add(c->B.scal + S_DTFIX, c->tape_dt + n, sizeof(double));
      snap_save(c, seg_stage(c, n - n0, s, ns), sidx, pre);
      states_copies(c, post, seg_qstar(c, n - n0, s, ns), true);
      if (s == 0) ext_save(c, seg_ext(c, n - n0, ns), post);
      bool fit = pre.full.empty() && post.full.empty();
      if (!fit) pre.run(c);
      stage<D>(c, s, sidx, 0, didx, b[s], cc[s], w[s], (double*)seg_qstar(c, n - n0, s, ns),
               seg_qstar_occ(c, n - n0, s, ns), false, fit ? pre.L : kNoCopies,
               fit ? post.L : kNoCopies);
      if (!fit) post.run(c);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint buffers (allocated on first use)
// ---------------------------------------------------------------------------
static mm_status adj_alloc(mm_ctx* c) {
  if (c->adj_ready) return MM_OK;
  const Params& P = c->P;
  size_t nc = P.NC, M = P.M, nv = P.dim + 2;
  Adj& A = c->A;
  memset(&A, 0, sizeof(A));
  hipError_t e = hipSuccess;
#define AA(p, n)                                     \
  if (e == hipSuccess) {                             \
    e = dalloc(c, &(p), (n));                        \
  }
  AA(A.lQ, M * 4 * nc); AA(A.lQs, M * 4 * nc); AA(A.lQn, M * 4 * nc);
  AA(A.lphis, nc); AA(A.lphin, nc);
  // one block, cleared at once each stage: lW, lal, lax, lay, lcx, lcy, lphi
  double* blk = nullptr;
  AA(blk, (M * 4 + 5 * M + 1) * nc);
  if (e == hipSuccess) {
    A.lW = blk;
    A.lal = blk + M * 4 * nc;
    A.lax = A.lal + M * nc;
    A.lay = A.lax + M * nc;
    A.lcx = A.lay + M * nc;
    A.lcy = A.lcx + M * nc;
    A.lphi = A.lcy + M * nc;
  }
  AA(A.lvx, nc); AA(A.lvy, nc);
  if (P.dim == 2) AA(A.lW2, M * 4 * nc);
  AA(A.linflow, 4);
  AA(A.lalpha, M * nc);
  (void)nv;
  AA(c->ctr_save, C_N); AA(c->scal_save, 8); AA(c->cons_save, CONS_N);
#undef AA
  if (e != hipSuccess) return fail(c, MM_ENOMEM, "adjoint buffers");
  c->adj_ready = true;
  return MM_OK;
}

// reverse of recorded step n: on entry A.lQ / A.lphi hold the adjoint of the
// state after step n (and A.lalpha that of its volume fractions), on exit
// that of the state before it
template <int D>
static void reverse_step(mm_ctx* c, int64_t n, bool with_alpha) {
  const Params& P = c->P;
  size_t nc = P.NC, M = P.M;
  double b[3], cc[3], w[3];
  int ns = rk_coefs(c->cfg, b, cc, w);
  dim3 g = cell_grid(c), bl = cell_block(c);
  dim3 gm(g.x, g.y, P.M);  // one material per slice
  Adj& A = c->A;
  int64_t rel = n - c->seg_n0;
  Copies z;
  z.fill0(A.lQn, M * 4 * nc * 8);
  z.fill0(A.lphin, nc * 8);
  z.fill0(A.lvx, nc * 8);
  z.fill0(A.lvy, nc * 8);
  z.run(c);
  int nfx0 = (P.nx + 1) * P.ny, nfx1 = P.nx * (P.ny + 1);
  for (int s = ns - 1; s >= 0; s--) {
    int sidx = stage_src(s), didx = stage_dst(s, ns);
    // phase 1: mixing and the geometry of the new level set, from the
    // snapshot that follows this stage and the stage's Q*
    const char* next;
    if (s + 1 < ns) next = seg_stage(c, rel, s + 1, ns);
    else if (n + 1 == c->tape_n) next = c->final_snap;
    else if (n + 1 < c->seg_n1) next = seg_stage(c, rel + 1, 0, ns);
    else next = c->ckpt[(n + 1) / c->tape_K];
    // with the snapshot's copies: the adjoints of the stage's output become
    // those of Q* and of the new level set, and the geometry adjoints start
    // from zero (lal, lax, lay, lcx, lcy)
    Copies c1;
    c1.add(A.lQs, A.lQ, M * 4 * nc * 8);
    c1.add(A.lphis, A.lphi, nc * 8);
    c1.fill0(A.lal, 5 * M * nc * 8);
    // the step's first reversed stage sets the recorded step size (grid
    // slice z = M of the mixing adjoint); it holds for all stages of the step
    if (s == ns - 1) c1.add(c->B.scal + S_DTFIX, c->tape_dt + n, sizeof(double));
    snap_load<D>(c, next, didx, &c1, false);
    A.Qstar = (double*)seg_qstar(c, rel, s, ns);
    A.occstar = seg_qstar_occ(c, rel, s, ns);
    LAUNCH(k_a_mix<D>, dim3(g.x, g.y, P.M + (s == ns - 1 ? 1 : 0)), bl, P, c->B, A);
    if (s == ns - 1 && with_alpha) LAUNCH(k_a_add_alpha, g, bl, P, c->B, A);
    LAUNCH(k_a_geom<D>, gm, bl, P, c->B, A, A.lphis);
    if (D == 2)
      LAUNCH(k_a_bc_ls2, lin_grid(((long)P.ny + P.nx + 2 * H) * 2 * H), dim3(256), P, A.lphis);
    else
      LAUNCH(k_a_bc_ls_x, lin_grid((long)P.ny * 2 * H), dim3(256), P, A.lphis);
    // phase 2: the stage's input with the states it read (kept by the
    // segment recompute); for s > 0 also the time-n state in buffer 0, the
    // velocity and the time-n level set
    Copies cp;
    if (s > 0) {
      SnapLayout L = snap_layout(P);
      const char* s0 = seg_stage(c, rel, 0, ns);
      cp.add(c->B.Q[0], s0 + L.q, M * (P.dim + 2) * nc * 8);
      cp.add(c->B.occ[0], s0 + L.occ, nc);
      ext_add(c, cp, seg_ext(c, rel, ns));
    }
    states_copies(c, cp, seg_qstar(c, rel, s, ns), false);
    // the adjoints of the stage's input from zero
    cp.fill0(A.lW, M * 4 * nc * 8);
    cp.fill0(A.lal, (5 * M + 1) * nc * 8);  // lal..lcy, lphi
    snap_load<D>(c, seg_stage(c, rel, s, ns), sidx, &cp, false);
    // with the update and (2D) the tile list of the stage's own level set
    LAUNCH(k_a_ls<D>, dim3(g.x, g.y, D == 2 ? 3 : 2), bl, P, c->B, A, b[s], cc[s], sidx);
    // at stage 0 with the velocity fill reversed in extra workgroups
    unsigned nfb = lin_grid(D == 2 ? nfx0 + nfx1 : nfx0).x;
    unsigned nvb = s == 0 ? lin_grid((long)P.nx * P.ny).x : 0;
    LAUNCH(k_a_flux<D>, dim3(nfb + nvb), dim3(256), P, c->B, A, sidx, cc[s], (int)nfb);
    if (s == 0) {
      for (int sw = 3; sw >= 0; sw--) LAUNCH(k_a_vext<D>, g, bl, P, c->B, A, sw);
    }
    // 2D: with the frames of the primitive states in grid slice z = 1
    LAUNCH(k_a_iface<D>, dim3(g.x, g.y, D == 2 ? 2 : 1), bl, P, c->B, A, sidx, cc[s],
           s == 0 ? 1 : 0);
    if (D == 1) LAUNCH(k_a_bc_W_x, lin_grid((long)P.ny * 2 * H * P.M), dim3(256), P, c->B, A);
    if (D == 2) {
      // tile-wise, on the tiles of the stage's own level set (its snapshot was
      // classified on loading); lW is read throughout, lW2 written
      cpy(c, A.lW2, A.lW, M * 4 * nc * 8);
      LAUNCH(k_a_ext_tiles, dim3(tile_grid(c).x, P.M), dim3(256), P, c->B, A, sidx);
      std::swap(A.lW, A.lW2);  // the written buffer holds the result
    } else {
      for (int sw = P.kext + 3; sw >= 0; sw--)
        LAUNCH(k_a_ext<D>, dim3(256), dim3(256), P, c->B, A, sidx, sw);
    }
    LAUNCH(k_a_real<D>, gm, bl, P, c->B, A, sidx);
    LAUNCH(k_a_geom<D>, gm, bl, P, c->B, A, A.lphi);
    // the frame's level-set adjoint goes to the inside cells here only at
    // the step's first stage; before, the next stage copies it along and
    // passes it on with its own (the pass is linear)
    // (2D with the finish of the step in the same launch)
    if (s == 0) {
      if (D == 2) {
        unsigned nfrb = lin_grid(((long)P.ny + P.nx + 2 * H) * 2 * H).x;
        LAUNCH(k_a_bc_ls2_finish, dim3(nfrb + lin_grid((long)P.nx * P.ny).x), dim3(256), P, A,
               (int)nfrb);
      } else {
        LAUNCH(k_a_bc_ls_x, lin_grid((long)P.ny * 2 * H), dim3(256), P, A.lphi);
      }
    }
  }
  if (D == 1) LAUNCH(k_a_finish, g, bl, P, A);
}

extern "C" mm_status mm_adjoint_step(mm_ctx* c, const double* lamQ_in, const double* lamPhi_in,
                                     const double* lamAlpha_in, double* lamQ_out,
                                     double* lamPhi_out, int32_t ptr_kind) {
  if (!c) return MM_EINVAL;
  if (ptr_kind != MM_HOST && ptr_kind != MM_DEVICE) return fail(c, MM_EINVAL, "bad ptr_kind");
  if (c->tape_K <= 0 || c->tape_rev <= 0)
    return fail(c, MM_ESTATE, "no recorded step left to reverse");
  if (c->tape_moved)
    return fail(c, MM_ENOTIMPL,
                "a recorded step moved conserved quantities between materials (stranded "
                "mixing sources or scale separation); the adjoint does not cover it");
  mm_status st = adj_alloc(c);
  if (st != MM_OK) return st;
  const Params& P = c->P;
  size_t plane = (size_t)P.nx * P.ny, nv = P.dim + 2;
  size_t nQ = (size_t)P.M * nv * plane, nA = (size_t)P.M * plane;
  Adj& A = c->A;
  SnapLayout L = snap_layout(P);
  // first reverse call: keep the forward state after the last recorded step;
  // every call: keep the counters, scalars and sums (restored at the end)
  Copies sv;
  if (c->tape_rev == c->tape_n) {
    HIP_OK(c, grow(c, &c->final_snap, &c->final_cap, L.bytes));
    snap_save(c, c->final_snap, 0, sv);
    sv.fill0(A.linflow, 4 * 8);
    sv.fill0(A.lQ, (size_t)P.M * 4 * P.NC * 8);
    sv.fill0(A.lphi, (size_t)P.NC * 8);
  }
  // (the saved copies still hold them right after another reverse call)
  if (!c->adj_clean || c->tape_rev == c->tape_n) {
    sv.add(c->ctr_save, c->B.ctr, C_N * sizeof(unsigned long long));
    sv.add(c->scal_save, c->B.scal, 8 * sizeof(double));
    sv.add(c->cons_save, c->B.cons, CONS_N * sizeof(double));
  }
  sv.run(c);
  c->adj_clean = false;
  // inputs (device copies of host arrays in the staging buffer)
  const double *dQ = lamQ_in, *dphi = lamPhi_in, *dal = lamAlpha_in;
  if (ptr_kind == MM_HOST && (lamQ_in || lamPhi_in || lamAlpha_in || lamQ_out || lamPhi_out)) {
    size_t need = (nQ + plane + nA) * sizeof(double);
    if (c->d_in_bytes < need) {
      if (c->d_in) (void)hipFree(c->d_in);
      c->d_in = nullptr;
      c->d_in_bytes = 0;
      if (hipMalloc(&c->d_in, need) != hipSuccess) return fail(c, MM_ENOMEM, "staging buffer");
      c->d_in_bytes = need;
    }
    double* q0 = c->d_in;
    double* p0 = q0 + nQ;
    double* a0 = p0 + plane;
    if (lamQ_in)
      HIP_OK(c, hipMemcpyAsync(q0, lamQ_in, nQ * 8, hipMemcpyHostToDevice, c->stream));
    if (lamPhi_in)
      HIP_OK(c, hipMemcpyAsync(p0, lamPhi_in, plane * 8, hipMemcpyHostToDevice, c->stream));
    if (lamAlpha_in)
      HIP_OK(c, hipMemcpyAsync(a0, lamAlpha_in, nA * 8, hipMemcpyHostToDevice, c->stream));
    dQ = lamQ_in ? q0 : nullptr;
    dphi = lamPhi_in ? p0 : nullptr;
    dal = lamAlpha_in ? a0 : nullptr;
    // the caller's arrays may be reused once this call returns
    if (lamQ_in || lamPhi_in || lamAlpha_in) HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  dim3 g = cell_grid(c), bl = cell_block(c);
  if (dQ || dphi || dal) {
    if (c->D == 2) LAUNCH(k_a_unpack<2>, g, bl, P, A, dQ, dphi, dal);
    else LAUNCH(k_a_unpack<1>, g, bl, P, A, dQ, dphi, dal);
  }
  int64_t n = c->tape_rev - 1;
  int64_t K = c->tape_K, n0 = (n / K) * K, n1 = n0 + K < c->tape_n ? n0 + K : c->tape_n;
  if (c->seg_n0 != n0) {
    double b[3], cc[3], w[3];
    int ns = rk_coefs(c->cfg, b, cc, w);
    HIP_OK(c, grow(c, &c->seg, &c->seg_cap, (size_t)(n1 - n0) * seg_step_bytes(c, ns)));
    if (c->D == 2) load_segment<2>(c, n0, n1);
    else load_segment<1>(c, n0, n1);
    c->seg_n0 = n0;
    c->seg_n1 = n1;
  }
  if (c->D == 2) reverse_step<2>(c, n, dal != nullptr);
  else reverse_step<1>(c, n, dal != nullptr);
  c->tape_rev--;
  // outputs
  if (lamQ_out || lamPhi_out) {
    double* oq = lamQ_out;
    double* op = lamPhi_out;
    if (ptr_kind == MM_HOST) {
      oq = c->d_in;
      op = c->d_in + nQ;
    }
    if (c->D == 2) LAUNCH(k_a_pack<2>, g, bl, P, A, oq, lamPhi_out ? op : nullptr);
    else LAUNCH(k_a_pack<1>, g, bl, P, A, oq, lamPhi_out ? op : nullptr);
    if (ptr_kind == MM_HOST) {
      if (lamQ_out) HIP_OK(c, hipMemcpyAsync(lamQ_out, oq, nQ * 8, hipMemcpyDeviceToHost, c->stream));
      if (lamPhi_out)
        HIP_OK(c, hipMemcpyAsync(lamPhi_out, op, plane * 8, hipMemcpyDeviceToHost, c->stream));
    }
  }
  // the forward state after the recorded run, and the diagnostics, as they were
  // counters as they were, but the mixing stamp (it only grows) and the tile
  // count (the tile list is rebuilt)
  static_assert(C_STAMP + 1 == C_NTILES, "counters restored in two ranges");
  Copies rs;
  rs.add(c->B.scal, c->scal_save, 8 * sizeof(double));
  rs.add(c->B.cons, c->cons_save, CONS_N * sizeof(double));
  rs.add(c->B.ctr, c->ctr_save, C_STAMP * sizeof(unsigned long long));
  rs.add(c->B.ctr + C_NTILES + 1, c->ctr_save + C_NTILES + 1,
         (C_N - C_NTILES - 1) * sizeof(unsigned long long));
  // (the forward tile list is rebuilt when next needed)
  if (c->D == 2) snap_load<2>(c, c->final_snap, 0, &rs, false);
  else snap_load<1>(c, c->final_snap, 0, &rs, false);
  c->tiles_stale = true;
  HIP_OK(c, hipGetLastError());
  c->adj_clean = true;
  // host outputs need the work done; otherwise the next call may queue
  // behind this one
  if (ptr_kind == MM_HOST && (lamQ_out || lamPhi_out)) HIP_OK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

extern "C" mm_status mm_adjoint_inflow(mm_ctx* c, double* out) {
  if (!c || !out) return MM_EINVAL;
  if (!c->adj_ready) {
    for (int v = 0; v < 4; v++) out[v] = 0.0;
    return MM_OK;
  }
  HIP_OK(c, hipMemcpyAsync(out, c->A.linflow, 4 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

extern "C" mm_status mm_tape_info(mm_ctx* c, int64_t* recorded, int64_t* remaining,
                                  double* dt) {
  if (!c) return MM_EINVAL;
  if (recorded) *recorded = c->tape_K > 0 ? c->tape_n : 0;
  if (remaining) *remaining = c->tape_K > 0 ? c->tape_rev : 0;
  if (dt && c->tape_K > 0 && c->tape_n > 0) {
    HIP_OK(c, hipMemcpyAsync(dt, c->tape_dt, c->tape_n * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  return MM_OK;
}
