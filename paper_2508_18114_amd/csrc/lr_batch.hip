// Host side of the batch entry points (lr_batch_*): planning, workspace
// layout and the launch sequence that integrates many independent
// trajectories with the persistent on-chip kernel.
//
// Spread schedule (the default): trajectories are sorted by step count
// (longest first, stable) and packed, in that order, into execution groups
// whose workgroups are co-resident (one cooperative launch per chunk of
// steps); groups run one after the other, so trajectories of similar length
// share a group and few workgroups idle.  Within a group every trajectory has
// its own barrier flags, so trajectories of different shapes and step counts
// proceed independently, and each result is bitwise that of the trajectory
// alone.
//
// Packed schedule (LR_BATCH_PACKED): every trajectory whose layer fits the
// packed kernel gets one workgroup of its own (lr_packed.hip); the packed
// trajectories of one kernel family (model kind 2 or not, arithmetic mode)
// go into one ordinary launch per chunk, largest work first, and the hardware
// fills each CU with as many as fit; the launch sequences of different
// families run concurrently on forked streams.  The others run in spread
// groups.
//
// Layer-split packed trajectories (LR_BATCH_PACKED_PARTS): each FP64 packed
// trajectory runs on P workgroups of the packed kernel (lr_packed.hip,
// lr_adaptive.hip), in co-resident groups of one cooperative launch per
// chunk, like the spread groups; the one-workgroup prologue forms the Gram
// terms of the initial state.

struct lr_batch {
  int n = 0;
  std::vector<lr_traj_t> tr;   // in execution order (see lr_batch_init)
  std::vector<int> pos;        // pos[i] = execution position of the caller's trajectory i
  std::vector<TrajDev> dev;
  std::vector<int> P, prt, rows;
  std::vector<size_t> lds, region, region_bytes;
  std::vector<int> wg_offset;  // first tilemap entry of each trajectory
  std::vector<char> packed;    // trajectory runs in the packed kernel
  std::vector<char> split;     // packed trajectory split over P[t] workgroups (layer ranges)
  bool graph_on = false;       // lr_batch_run captures its launch sequence once and replays it
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool adaptive = false;       // packed trajectories take adaptive Dormand-Prince steps
  double rtol = 0.0, atol = 0.0;
  size_t off_ad = 0;           // AdaptDev descriptors (adaptive batches)
  std::vector<lrk::AdaptDev> ad;
  size_t off_trajs = 0, off_tilemap = 0, total = 0;
  int total_wg = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  // packed groups after the first run concurrently on streams of their own
  // (forked from and joined back into `stream` by events)
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_ev;  // [0]: fork; [1 + i]: join of aux[i]
  struct Group {
    int begin, end, wgs, rows, ge, prec;
    size_t lds;
    int64_t max_steps, chunk;
    int packed, kp;
    int nm;     // packed group of the normal-mode model (its own kernels)
    int gm;     // packed: Gram terms on the vector ALU (-1) or matrix-core mode (0 FP64, 1 FP32, 2 BF16x3)
    int slots;  // packed matrix-core modes: output tiles per wave
    int split;  // packed, layer-split trajectories (cooperative launch, wgs = sum of the parts)
  };
  bool mfma64 = false;  // LR_BATCH_PACKED_MFMA64
  std::vector<Group> groups;
  bool prof = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs of timed chunk launches
  int64_t n_ev = 0;
};

namespace {

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Persistent configuration of one shape: layers per workgroup, register rows.
bool persist_config(const lr_model_t& m, int M, int layers, int& prt, int& P, int& rows, size_t& lds) {
  const int L = m.d_q * m.d_f;
  const int NG = lrk::kPW / M;
  prt = 1;
  if (const char* e = std::getenv("LR_PERSIST_LAYERS")) prt = std::atoi(e);
  if (layers > 0) prt = layers;
  if (prt < 1) prt = 1;
  if (prt > m.d_r) prt = m.d_r;
  while (prt > 1 && ((prt * L + NG - 1) / NG > lrk::kMaxRowsPerThread ||
                     lrk::persist_lds_bytes(prt, L, M, (m.d_r + prt - 1) / prt) > lrk::kPersistLdsMax))
    --prt;
  P = (m.d_r + prt - 1) / prt;
  while (P > 256 && prt < m.d_r) {  // one cooperative launch must hold the trajectory
    ++prt;
    P = (m.d_r + prt - 1) / prt;
  }
  rows = ((prt * L + NG - 1) / NG <= 2) ? 2 : 3;
  lds = lrk::persist_lds_bytes(prt, L, M, P);
  return (prt * L + NG - 1) / NG <= lrk::kMaxRowsPerThread && lds <= lrk::kPersistLdsMax && P <= 256;
}

int check_model(const lr_model_t& m, int M, int precision) {
  if (m.d_q < 2 || m.d_r < 1 || m.d_f < 1) return LR_ERR_ARG;
  if (m.kind != LR_MODEL_DUFFING && m.kind != LR_MODEL_TRANSMON && m.kind != LR_MODEL_NORMAL) return LR_ERR_ARG;
  if (m.kind == LR_MODEL_NORMAL) {
    if (precision != LR_FP64) return LR_ERR_ARG;
    for (double x : m.S)
      if (!std::isfinite(x)) return LR_ERR_ARG;
  }
  if (m.kind == LR_MODEL_TRANSMON || m.kind == LR_MODEL_NORMAL) {
    if (m.d_q > LR_MAX_DQ) return LR_ERR_ARG;
    double big = 0.0;
    for (int i = 0; i < m.d_q * m.d_q; ++i) {
      if (!std::isfinite(m.n_t[i])) return LR_ERR_ARG;
      big = std::max(big, std::fabs(m.n_t[i]));
    }
    for (int i = 0; i < m.d_q; ++i) {
      if (!std::isfinite(m.E_t[i])) return LR_ERR_ARG;
      for (int j = 0; j < i; ++j)
        if (std::fabs(m.n_t[i * m.d_q + j] - m.n_t[j * m.d_q + i]) > 1e-12 * big) return LR_ERR_ARG;
    }
  }
  const long long N = (long long)m.d_q * m.d_r * m.d_f;
  if (N > (1LL << 26)) return LR_ERR_ARG;
  if (M < 1 || M > LR_MAX_M || M > N) return LR_ERR_ARG;
  if (precision != LR_FP64 && precision != LR_FP32 && precision != LR_BF16X3) return LR_ERR_ARG;
  const double vals[] = {m.w_q, m.alpha, m.w_r, m.w_f, m.g, m.G, m.kappa_f, m.gamma_1};
  for (double x : vals)
    if (!std::isfinite(x)) return LR_ERR_ARG;
  if (m.kappa_f < 0.0 || m.gamma_1 < 0.0) return LR_ERR_ARG;
  return LR_OK;
}

const void* persist_fn(int rows, int ge, int prec, bool prologue = false) {
  return lrk::persist_kernel(rows, ge, prologue, prec);
}

int batch_init(lr_batch_t** out, const lr_traj_t* trajs, int32_t n, int32_t flags, bool adaptive, double rtol,
               double atol);

}  // namespace

extern "C" {

int lr_batch_init(lr_batch_t** out, const lr_traj_t* trajs, int32_t n) {
  return lr_batch_init_ex(out, trajs, n, 0);
}

int lr_batch_init_ex(lr_batch_t** out, const lr_traj_t* trajs, int32_t n, int32_t flags) {
  return batch_init(out, trajs, n, flags, false, 0.0, 0.0);
}

int lr_batch_init_adaptive(lr_batch_t** out, const lr_traj_t* trajs, int32_t n, double rtol, double atol) {
  return lr_batch_init_adaptive_ex(out, trajs, n, 0, rtol, atol);
}

int lr_batch_init_adaptive_ex(lr_batch_t** out, const lr_traj_t* trajs, int32_t n, int32_t flags, double rtol,
                              double atol) {
  if (!(rtol > 0.0) || !(atol > 0.0) || !std::isfinite(rtol) || !std::isfinite(atol)) return LR_ERR_ARG;
  if (flags & ~(LR_BATCH_PACKED | LR_BATCH_PACKED_PARTS(0xff))) return LR_ERR_ARG;
  return batch_init(out, trajs, n, flags | LR_BATCH_PACKED, true, rtol, atol);
}

int lr_batch_adaptive_stats(lr_batch_t* b, int64_t* accepted, int64_t* rejected) {
  if (!b) return LR_ERR_ARG;
  if (!b->adaptive) return LR_ERR_STATE;
  if (!b->ws) return LR_ERR_STATE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LR_ERR_HIP;
  for (int i = 0; i < b->n; ++i) {
    int64_t c[2] = {0, 0};
    if (hipMemcpy(c, b->ad[b->pos[i]].cnt, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return LR_ERR_HIP;
    if (accepted) accepted[i] = c[0];
    if (rejected) rejected[i] = c[1];
  }
  return LR_OK;
}

}  // extern "C"

namespace {
int batch_init(lr_batch_t** out, const lr_traj_t* trajs, int32_t n, int32_t flags, bool adaptive, double rtol,
               double atol) {
  if (!out || !trajs || n < 1) return LR_ERR_ARG;
  if (flags & ~(LR_BATCH_PACKED | LR_BATCH_PACKED_MFMA64 | LR_BATCH_SPREAD_LAYERS(0xff) | LR_BATCH_PACKED_PARTS(0xff)))
    return LR_ERR_ARG;
  const int parts = (flags >> 16) & 0xff;
  *out = nullptr;
  lr_batch* b = new (std::nothrow) lr_batch();
  if (!b) return LR_ERR_OOM;
  b->n = n;
  b->adaptive = adaptive;
  b->mfma64 = (flags & LR_BATCH_PACKED_MFMA64) != 0;
  b->rtol = rtol;
  b->atol = atol;
  auto packs = [&](const lr_traj_t& x) {
    const long long LM = (long long)x.model.d_q * x.model.d_f * x.M;
    // reduced arithmetic: kinds 0 and 1 (matrix-core Gram terms); adaptive steps: FP64
    const bool prec_ok = x.precision == LR_FP64 || (!adaptive && x.model.kind != LR_MODEL_NORMAL &&
                                                   (x.precision == LR_FP32 || x.precision == LR_BF16X3));
    if (!((flags & LR_BATCH_PACKED) && prec_ok && x.M >= 1 && x.M <= lrk::kMaxM && LM >= 1 &&
          LM <= lrk::kTMaxLM && x.model.d_r >= 1 && x.model.d_r <= (1 << 20)))
      return false;
    const int dmax = std::max(std::max(x.model.d_q, x.model.d_r), x.model.d_f);
    return lrk::packed_lds_elems(x.model.d_q * x.model.d_f, x.M, dmax, x.model.kind) * sizeof(double2) <=
           lrk::kPackedLdsMax;
  };
  auto work = [&](const lr_traj_t& x) {
    return (double)x.nsteps * x.model.d_q * x.model.d_r * x.model.d_f * x.M;
  };
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  // packed trajectories first, largest work first; then one precision mode
  // per spread group (kernel variants differ by it), longest first
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const bool px = packs(trajs[x]), py = packs(trajs[y]);
    if (px != py) return px;
    if (px) {  // kernel families together: kind 2 last, then by arithmetic mode
      const bool nx = trajs[x].model.kind == LR_MODEL_NORMAL, ny = trajs[y].model.kind == LR_MODEL_NORMAL;
      if (nx != ny) return ny;
      if (trajs[x].precision != trajs[y].precision) return trajs[x].precision < trajs[y].precision;
      return work(trajs[x]) > work(trajs[y]);
    }
    if (trajs[x].precision != trajs[y].precision) return trajs[x].precision < trajs[y].precision;
    return trajs[x].nsteps > trajs[y].nsteps;
  });
  b->tr.resize(n);
  b->pos.resize(n);
  b->packed.resize(n);
  b->split.resize(n);
  for (int k = 0; k < n; ++k) {
    b->tr[k] = trajs[order[k]];
    b->pos[order[k]] = k;
    b->packed[k] = packs(b->tr[k]);
    b->split[k] = b->packed[k] && parts >= 2 && b->tr[k].precision == LR_FP64;
  }
  b->dev.resize(n);
  b->P.resize(n);
  b->prt.resize(n);
  b->rows.resize(n);
  b->lds.resize(n);
  b->region.resize(n);
  b->region_bytes.resize(n);
  b->wg_offset.resize(n);
  if (adaptive)  // every trajectory must take the packed kernel
    for (int k = 0; k < n; ++k)
      if (!b->packed[k]) {
        delete b;
        return LR_ERR_ARG;
      }
  for (int k = 0; k < n; ++k)  // the eigenbasis models run packed
    if (b->tr[k].model.kind != LR_MODEL_DUFFING && !b->packed[k]) {
      delete b;
      return LR_ERR_ARG;
    }
  const size_t a = 256;
  size_t o = 0;
  b->off_trajs = o;
  o = align_up(o + sizeof(TrajDev) * (size_t)n, a);
  b->off_ad = o;
  if (adaptive) o = align_up(o + sizeof(lrk::AdaptDev) * (size_t)n, a);
  int wg = 0;
  for (int t = 0; t < n; ++t) {
    const lr_traj_t& x = b->tr[t];
    int e = check_model(x.model, x.M, x.precision);
    if (!e) e = check_pulse(&x.pulse);
    if (!e && (!x.d_B || !std::isfinite(x.t0) || !(x.dt > 0.0) || !std::isfinite(x.dt) || x.nsteps < 0 ||
               x.obs_stride < 0 || (x.obs_stride > 0 && !x.d_obs) || x.step0 < 0))
      e = LR_ERR_ARG;
    if (!e && b->packed[t]) {
      b->prt[t] = 0;
      b->P[t] = b->split[t] ? std::min(parts, x.model.d_r) : 1;
      b->rows[t] = 0;
      b->lds[t] = lrk::packed_lds_elems(x.model.d_q * x.model.d_f, x.M,
                                        std::max(std::max(x.model.d_q, x.model.d_r), x.model.d_f), x.model.kind) *
                  sizeof(double2);
    } else if (!e && !persist_config(x.model, x.M, (flags >> 8) & 0xff, b->prt[t], b->P[t], b->rows[t], b->lds[t])) {
      e = LR_ERR_ARG;
    }
    if (e) {
      delete b;
      return e;
    }
    b->wg_offset[t] = wg;
    wg += b->P[t];
  }
  b->total_wg = wg;
  b->off_tilemap = o;
  o = align_up(o + sizeof(int2) * (size_t)wg, a);
  for (int t = 0; t < n; ++t) {
    const lr_traj_t& x = b->tr[t];
    const size_t N = (size_t)x.model.d_q * x.model.d_r * x.model.d_f;
    const size_t nm = N * x.M * sizeof(double2), npe = 3 * (size_t)x.M * x.M * sizeof(double2);
    const size_t P = b->P[t];
    size_t r = 0;
    if (b->packed[t]) {
      for (int k = 0; k < 4; ++k) r = align_up(r + nm, a);  // Bb, S0, S1, acc
      r = align_up(r + 2 * (size_t)x.M * x.M * sizeof(double2), a);  // W
      if (adaptive) {
        r = align_up(r + 7 * nm, a);                       // k_1 .. k_7
        r = align_up(r + 64, a);                           // t, h, counters
      }
      if (b->split[t]) {
        const size_t spe = lrk::split_npe(x.M, x.model.kind) * sizeof(double2);
        r = align_up(r + P * spe, a);                      // PART
        r = align_up(r + spe + P * sizeof(double), a);     // RED, one value per part
        r = align_up(r + P * lrk::kFlagStride * 4, a);     // flagA
        r = align_up(r + 2 * P * lrk::kFlagStride * 4, a); // flagB, flagC
      }
      r = align_up(r + 64, a);                             // step, fail_step, fro2, status, abort
      b->region[t] = o;
      b->region_bytes[t] = r;
      o += r;
      continue;
    }
    r = align_up(r + nm, a);                               // Bb
    r = align_up(r + 2 * nm, a);                           // SP
    r = align_up(r + 2 * P * npe, a);                      // PART
    r = align_up(r + 2 * npe, a);                          // RED
    r = align_up(r + P * lrk::kFlagStride * 4, a);         // flagA
    r = align_up(r + P * lrk::kFlagStride * 4, a);         // flagB
    r = align_up(r + 64, a);                               // step, fail_step, fro2, status, abort
    b->region[t] = o;
    b->region_bytes[t] = r;
    o += r;
  }
  b->total = o;
  *out = b;
  return LR_OK;
}
}  // namespace

extern "C" {

size_t lr_batch_workspace_bytes(const lr_batch_t* b) { return b ? b->total : 0; }

int lr_batch_bind(lr_batch_t* b, void* d_ws, size_t bytes, void* stream) {
  if (!b || !d_ws) return LR_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return LR_ERR_ARG;
  if (bytes < b->total) return LR_ERR_OOM;
  b->ws = static_cast<char*>(d_ws);
  b->stream = static_cast<hipStream_t>(stream);
  b->ad.assign(b->adaptive ? b->n : 0, lrk::AdaptDev{});
  const size_t a = 256;
  std::vector<int2> tmap((size_t)b->total_wg);
  for (int t = 0; t < b->n; ++t) {
    const lr_traj_t& x = b->tr[t];
    const lr_model_t& m = x.model;
    const size_t N = (size_t)m.d_q * m.d_r * m.d_f;
    const size_t nm = N * x.M * sizeof(double2), npe = 3 * (size_t)x.M * x.M * sizeof(double2);
    const size_t P = b->P[t];
    char* base = b->ws + b->region[t];
    size_t r = 0;
    TrajDev& v = b->dev[t];
    v = TrajDev{};
    v.d_q = m.d_q; v.d_r = m.d_r; v.d_f = m.d_f; v.M = x.M;
    v.N = (int)N; v.L = m.d_q * m.d_f; v.ntiles = 0; v.obs_stride = x.obs_stride;
    v.nsteps = x.nsteps;
    v.w_q = m.w_q; v.alpha = m.alpha; v.w_r = m.w_r; v.w_f = m.w_f;
    v.g = m.g; v.G = m.G; v.kappa = m.kappa_f; v.gamma = m.gamma_1;
    v.mkind = m.kind;
    if (m.kind == LR_MODEL_TRANSMON || m.kind == LR_MODEL_NORMAL) {
      for (int i = 0; i < m.d_q; ++i) v.Et[i] = m.E_t[i];
      for (int i = 0; i < m.d_q * m.d_q; ++i) v.ntq[i] = m.n_t[i];
    }
    if (m.kind == LR_MODEL_NORMAL) {  // s_21 .. s_24; mu_l, mu_u, nu_l, nu_u (supplement S2.D)
      for (int i = 0; i < 4; ++i) v.nm[i] = m.S[4 + i];
      v.nm[4] = m.S[2] - m.S[1];
      v.nm[5] = m.S[3] - m.S[0];
      v.nm[6] = m.S[6] - m.S[5];
      v.nm[7] = m.S[7] - m.S[4];
    }
    set_pulse(v, &x.pulse);
    v.t0 = x.t0;
    v.dt = x.dt;
    v.step_base = x.step0;
    v.prec = x.precision;
    if (b->packed[t]) {
      v.Bb = reinterpret_cast<double2*>(base + r);      r = align_up(r + nm, a);
      v.S0 = reinterpret_cast<double2*>(base + r);      r = align_up(r + nm, a);
      v.S1 = reinterpret_cast<double2*>(base + r);      r = align_up(r + nm, a);
      v.acc = reinterpret_cast<double2*>(base + r);     r = align_up(r + nm, a);
      v.W = reinterpret_cast<double2*>(base + r);       r = align_up(r + 2 * (size_t)x.M * x.M * sizeof(double2), a);
      if (b->adaptive) {
        lrk::AdaptDev& d = b->ad[t];
        d.rtol = b->rtol;
        d.atol = b->atol;
        d.K = reinterpret_cast<double2*>(base + r);     r = align_up(r + 7 * nm, a);
        d.st = reinterpret_cast<double*>(base + r);
        d.cnt = reinterpret_cast<int64_t*>(base + r + 16);
        r = align_up(r + 64, a);
      }
      v.P = 0;
      v.rt = 0;
      if (b->split[t]) {
        const int spn = lrk::split_npe(x.M, m.kind);
        const size_t spe = (size_t)spn * sizeof(double2);
        v.PART = reinterpret_cast<double2*>(base + r);  r = align_up(r + P * spe, a);
        v.RED = reinterpret_cast<double2*>(base + r);   r = align_up(r + spe + P * sizeof(double), a);
        v.flagA = reinterpret_cast<uint32_t*>(base + r); r = align_up(r + P * lrk::kFlagStride * 4, a);
        v.flagB = reinterpret_cast<uint32_t*>(base + r); r = align_up(r + 2 * P * lrk::kFlagStride * 4, a);
        v.P = (int)P;
        v.npe = spn;
      }
      if (r + 64 > b->region_bytes[t]) return LR_ERR_STATE;  // layout of lr_batch_init_ex
      v.step = reinterpret_cast<int64_t*>(base + r);
      v.fail_step = reinterpret_cast<int64_t*>(base + r + 8);
      v.fro2 = reinterpret_cast<double*>(base + r + 16);
      v.status = reinterpret_cast<int32_t*>(base + r + 24);
      v.abort_flag = reinterpret_cast<uint32_t*>(base + r + 28);
      v.obs = x.obs_stride > 0 ? x.d_obs : nullptr;
      for (int w = 0; w < (int)P; ++w) tmap[(size_t)b->wg_offset[t] + w] = make_int2(t, w);
      continue;
    }
    v.Bb = reinterpret_cast<double2*>(base + r);        r = align_up(r + nm, a);
    v.SP = reinterpret_cast<double2*>(base + r);        r = align_up(r + 2 * nm, a);
    v.PART = reinterpret_cast<double2*>(base + r);      r = align_up(r + 2 * P * npe, a);
    v.RED = reinterpret_cast<double2*>(base + r);       r = align_up(r + 2 * npe, a);
    v.flagA = reinterpret_cast<uint32_t*>(base + r);    r = align_up(r + P * lrk::kFlagStride * 4, a);
    v.flagB = reinterpret_cast<uint32_t*>(base + r);    r = align_up(r + P * lrk::kFlagStride * 4, a);
    if (r + 64 > b->region_bytes[t]) return LR_ERR_STATE;  // layout of lr_batch_init_ex
    v.step = reinterpret_cast<int64_t*>(base + r);
    v.fail_step = reinterpret_cast<int64_t*>(base + r + 8);
    v.fro2 = reinterpret_cast<double*>(base + r + 16);
    v.status = reinterpret_cast<int32_t*>(base + r + 24);
    v.abort_flag = reinterpret_cast<uint32_t*>(base + r + 28);
    v.obs = x.obs_stride > 0 ? x.d_obs : nullptr;
    v.P = (int)P;
    v.rt = b->prt[t];
    v.npe = 3 * x.M * x.M;
    v.prec = x.precision;
    for (int w = 0; w < (int)P; ++w) tmap[(size_t)b->wg_offset[t] + w] = make_int2(t, w);
  }
  hipError_t e1 = hipMemcpyAsync(b->ws + b->off_trajs, b->dev.data(), sizeof(TrajDev) * (size_t)b->n,
                                 hipMemcpyHostToDevice, b->stream);
  hipError_t e2 = hipMemcpyAsync(b->ws + b->off_tilemap, tmap.data(), sizeof(int2) * tmap.size(),
                                 hipMemcpyHostToDevice, b->stream);
  hipError_t e4 = hipSuccess;
  if (b->adaptive)
    e4 = hipMemcpyAsync(b->ws + b->off_ad, b->ad.data(), sizeof(lrk::AdaptDev) * b->ad.size(), hipMemcpyHostToDevice,
                        b->stream);
  hipError_t e3 = hipStreamSynchronize(b->stream);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) return LR_ERR_HIP;

  // execution groups of co-resident workgroups
  int dev_id = 0, ncu = 0;
  if (hipGetDevice(&dev_id) != hipSuccess) return LR_ERR_HIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess) return LR_ERR_HIP;
  size_t max_lds = 0, max_lds_packed = 0;
  for (int t = 0; t < b->n; ++t) {
    size_t& m = b->packed[t] ? max_lds_packed : max_lds;
    m = std::max(m, b->lds[t]);
  }
  // every packed kernel (one-workgroup chunk and prologue, layer-split chunk; fixed-step and adaptive;
  // kinds 0/1 and kind 2) may take the largest packed footprint
  if (max_lds_packed > 0)
    for (int kp : lrk::kPackedKP)
      for (int nm = 0; nm < 2; ++nm) {
        const void* fns[] = {lrk::packed_kernel(kp, false, nm != 0), lrk::packed_kernel(kp, true, nm != 0),
                             lrk::dp5_kernel(kp, false, nm != 0),    lrk::dp5_kernel(kp, true, nm != 0),
                             lrk::packed_split_kernel(kp, nm != 0),  lrk::dp5_split_kernel(kp, nm != 0)};
        for (const void* fn : fns)
          if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_packed) != hipSuccess)
            return LR_ERR_HIP;
      }
  for (int gm = 0; gm <= 2; ++gm)  // the matrix-core Gram kernels of the packed schedule
    for (int slots = 2; slots <= 3; ++slots)
      for (int pro = 0; pro < 2; ++pro)
        if (max_lds_packed > 0 && hipFuncSetAttribute(lrk::packed_kernel(0, pro != 0, false, gm, slots),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      (int)max_lds_packed) != hipSuccess)
          return LR_ERR_HIP;
  for (int prec = 0; prec <= 2; ++prec)
    for (int rows = 2; rows <= 3; ++rows)
      for (int ge = 1; ge <= 2; ++ge)
        for (int pro = 0; pro < 2; ++pro)
          if (hipFuncSetAttribute(persist_fn(rows, ge, prec, pro != 0), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)max_lds) != hipSuccess)
            return LR_ERR_HIP;
  auto capacity = [&](int rows, int ge, int prec, size_t lds) -> int {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_fn(rows, ge, prec), lrk::kPW, lds) !=
        hipSuccess)
      return 0;
    return per_cu * ncu;
  };
  b->groups.clear();
  int t = 0;
  while (t < b->n && b->packed[t]) {  // one launch per chunk holds every packed trajectory of a kernel family
    const int nm = b->tr[t].model.kind == LR_MODEL_NORMAL, prec = b->tr[t].precision;
    if (b->split[t]) {  // layer-split trajectories: co-resident groups of one kernel family
      lr_batch::Group g{t, t, 0, 0, 0, prec, 0, 0, 0, 1, 2, nm, -1, 2, 1};
      while (t < b->n && b->split[t] && (b->tr[t].model.kind == LR_MODEL_NORMAL) == (nm != 0)) {
        const int kp = std::max(g.kp, lrk::packed_kp(b->tr[t].M, b->tr[t].model.kind));
        const size_t lds = std::max(g.lds, b->lds[t]);
        const void* fn = b->adaptive ? lrk::dp5_split_kernel(kp, nm != 0) : lrk::packed_split_kernel(kp, nm != 0);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, lrk::kTW, lds) != hipSuccess) return LR_ERR_HIP;
        if (g.wgs + b->P[t] > per_cu * ncu) {
          if (g.end == g.begin) return LR_ERR_ARG;  // a single trajectory that cannot be co-resident
          break;
        }
        g.kp = kp;
        g.lds = lds;
        g.wgs += b->P[t];
        g.max_steps = std::max(g.max_steps, b->tr[t].nsteps);
        const int64_t s = b->tr[t].obs_stride;
        if (s > 0) g.chunk = g.chunk ? gcd64(g.chunk, s) : s;
        g.end = ++t;
      }
      if (g.chunk == 0) g.chunk = 4096;
      b->groups.push_back(g);
      continue;
    }
    const int gm = nm ? -1 : (prec == LR_FP64 ? (b->mfma64 && !b->adaptive ? 0 : -1) : prec);
    lr_batch::Group g{t, t, 0, 0, 0, prec, 0, 0, 0, 1, 2, nm, gm, 2, 0};
    // one launch for the family, sized by its largest LDS footprint (launches split by footprint
    // class, in order on one stream or concurrently on two, measured slower on mixed batches)
    while (t < b->n && b->packed[t] && !b->split[t] && (b->tr[t].model.kind == LR_MODEL_NORMAL) == (nm != 0) &&
           b->tr[t].precision == prec) {
      g.kp = std::max(g.kp, lrk::packed_kp(b->tr[t].M, b->tr[t].model.kind));
      g.slots = std::max(g.slots, lrk::mg_slots(b->tr[t].M));
      g.lds = std::max(g.lds, b->lds[t]);
      g.wgs += 1;
      g.max_steps = std::max(g.max_steps, b->tr[t].nsteps);
      const int64_t s = b->tr[t].obs_stride;
      if (s > 0) g.chunk = g.chunk ? gcd64(g.chunk, s) : s;
      g.end = ++t;
    }
    if (g.chunk == 0) g.chunk = 4096;
    b->groups.push_back(g);
  }
  {  // one forked stream per packed kernel family after the first (default priority)
    int npk = 0, prev = -1;
    for (const auto& g : b->groups)
      if (g.packed && !g.split && g.nm * 4 + g.prec != prev) {
        ++npk;
        prev = g.nm * 4 + g.prec;
      }
    while ((int)b->aux.size() < npk - 1) {
      hipStream_t sx = nullptr;
      if (hipStreamCreateWithFlags(&sx, hipStreamNonBlocking) != hipSuccess) return LR_ERR_HIP;
      b->aux.push_back(sx);
    }
    while (b->aux_ev.size() < b->aux.size() + 1) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return LR_ERR_HIP;
      b->aux_ev.push_back(e);
    }
  }
  while (t < b->n) {
    lr_batch::Group g{t, t, 0, 2, 1, b->tr[t].precision, 0, 0, 0, 0, 0, 0, -1, 2, 0};
    while (t < b->n) {
      if (b->tr[t].precision != g.prec) break;
      const int rows = std::max(g.rows, b->rows[t]);
      const int ge = std::max(g.ge, lrk::persist_ge(b->tr[t].M));
      const size_t lds = std::max(g.lds, b->lds[t]);
      const int cap = capacity(rows, ge, g.prec, lds);
      if (g.wgs + b->P[t] > cap) {
        if (g.end == g.begin) return LR_ERR_ARG;  // a single trajectory that cannot be co-resident
        break;
      }
      g.rows = rows;
      g.ge = ge;
      g.lds = lds;
      g.wgs += b->P[t];
      g.max_steps = std::max(g.max_steps, b->tr[t].nsteps);
      const int64_t s = b->tr[t].obs_stride;
      if (s > 0) g.chunk = g.chunk ? gcd64(g.chunk, s) : s;
      g.end = ++t;
    }
    if (g.chunk == 0) g.chunk = 4096;
    b->groups.push_back(g);
  }
  return LR_OK;
}

namespace {
void drop_graph(lr_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}
int enqueue(lr_batch* b);
}  // namespace

int lr_batch_graph(lr_batch_t* b, int32_t on) {
  if (!b) return LR_ERR_ARG;
  if (!b->ws) return LR_ERR_STATE;
  drop_graph(b);
  b->graph_on = false;
  if (!on) return LR_OK;
  if (!b->stream) return LR_ERR_STATE;  // the null stream cannot be captured
  for (int t = 0; t < b->n; ++t)
    if (!b->packed[t] || b->split[t]) return LR_ERR_STATE;  // cooperative launches are not captured
  b->graph_on = true;
  return LR_OK;
}

int lr_batch_run(lr_batch_t* b) {
  if (!b) return LR_ERR_ARG;
  if (!b->ws) return LR_ERR_STATE;
  if (!b->graph_on) return enqueue(b);
  if (!b->gexec) {
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LR_ERR_HIP;
    const int e = enqueue(b);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &g);
    if (e != LR_OK || ec != hipSuccess) {
      if (ec == hipSuccess && g) (void)hipGraphDestroy(g);
      return e != LR_OK ? e : LR_ERR_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(b);
      return LR_ERR_HIP;
    }
  }
  return hipGraphLaunch(b->gexec, b->stream) == hipSuccess ? LR_OK : LR_ERR_HIP;
}

}  // extern "C"

namespace {
int enqueue(lr_batch* b) {
  TrajDev* trajs = reinterpret_cast<TrajDev*>(b->ws + b->off_trajs);
  const int2* tmap = reinterpret_cast<const int2*>(b->ws + b->off_tilemap);
  hipLaunchKernelGGL(lrk::k_reset, dim3((b->n + 63) / 64), dim3(64), 0, b->stream, trajs, b->n);
  hipLaunchKernelGGL(lrk::k_reset_persist, dim3(b->n), dim3(256), 0, b->stream, trajs, b->n);
  const lrk::AdaptDev* ads = reinterpret_cast<const lrk::AdaptDev*>(b->ws + b->off_ad);
  if (b->adaptive)
    hipLaunchKernelGGL(lrk::k_dp5_reset, dim3((b->n + 63) / 64), dim3(64), 0, b->stream, trajs, ads, b->n);
  for (int t = 0; t < b->n; ++t) {
    const TrajDev& v = b->dev[t];
    long long e = (long long)v.N * v.M;
    const int grid = (int)std::min<long long>((e + lrk::kWG - 1) / lrk::kWG, 4096);
    hipLaunchKernelGGL(lrk::k_to_internal, dim3(grid), dim3(lrk::kWG), 0, b->stream, trajs, t,
                       reinterpret_cast<const double2*>(b->tr[t].d_B), v.Bb);
  }
  if (hipGetLastError() != hipSuccess) return LR_ERR_HIP;
  // packed kernel families run concurrently, the first on the batch stream and each further one on a
  // forked stream
  int nfam = 0, prev_fam = -1;
  std::vector<int> joins;
  // join the forked streams back into the batch stream (before any spread group: its cooperative
  // launch must find the chip free of packed work, or its group barriers could wait on workgroups
  // that cannot be resident yet)
  auto join_all = [&]() -> int {
    for (int i : joins) {
      if (hipEventRecord(b->aux_ev[1 + i], b->aux[i]) != hipSuccess) return LR_ERR_HIP;
      if (hipStreamWaitEvent(b->stream, b->aux_ev[1 + i], 0) != hipSuccess) return LR_ERR_HIP;
    }
    joins.clear();
    return LR_OK;
  };
  for (const auto& g : b->groups) {
    const TrajDev* gtr = trajs;
    const int2* gmap = tmap + b->wg_offset[g.begin];
    hipStream_t gs = b->stream;
    if (!g.packed || g.split)
      if (int e = join_all()) return e;
    if (g.packed && !g.split) {
      const int fam = g.nm * 4 + g.prec;
      if (fam != prev_fam) {
        ++nfam;
        prev_fam = fam;
        if (nfam > 1 && nfam - 2 < (int)b->aux.size()) {  // fork
          if (nfam == 2 && hipEventRecord(b->aux_ev[0], b->stream) != hipSuccess) return LR_ERR_HIP;
          if (hipStreamWaitEvent(b->aux[nfam - 2], b->aux_ev[0], 0) != hipSuccess) return LR_ERR_HIP;
          joins.push_back(nfam - 2);
        }
      }
      if (nfam > 1 && nfam - 2 < (int)b->aux.size()) gs = b->aux[nfam - 2];
    }
    auto launch = [&](int prologue, int64_t step0, int64_t nchunk) -> int {
      void* args[] = {(void*)&gtr, (void*)&gmap, (void*)&step0, (void*)&nchunk};
      int64_t k = -1;
      if (b->prof && !b->graph_on && !prologue && b->n_ev < LR_PROFILE_MAX) {
        while ((int64_t)b->ev.size() < 2 * (b->n_ev + 1)) {
          hipEvent_t e;
          if (hipEventCreate(&e) != hipSuccess) return LR_ERR_HIP;
          b->ev.push_back(e);
        }
        k = b->n_ev++;
        (void)hipEventRecord(b->ev[2 * k], gs);
      }
      hipError_t err;
      if (g.split) {  // one-workgroup prologue; chunks cooperative over the parts (flags zeroed first)
        const TrajDev* ptr = trajs + g.begin;
        const lrk::AdaptDev* aptr = ads + g.begin;
        const int ntr = g.end - g.begin;
        if (prologue) {
          void* pargs_a[] = {(void*)&ptr, (void*)&aptr, (void*)&step0, (void*)&nchunk};
          void* pargs_p[] = {(void*)&ptr, (void*)&step0, (void*)&nchunk};
          err = b->adaptive ? hipLaunchKernel(lrk::dp5_kernel(g.kp, true, g.nm != 0), dim3(ntr), dim3(lrk::kTW),
                                              pargs_a, g.lds, gs)
                            : hipLaunchKernel(lrk::packed_kernel(g.kp, true, g.nm != 0), dim3(ntr), dim3(lrk::kTW),
                                              pargs_p, g.lds, gs);
        } else {
          hipLaunchKernelGGL(lrk::k_reset_split, dim3(ntr), dim3(256), 0, gs, ptr, ntr);
          void* sargs_a[] = {(void*)&gtr, (void*)&ads, (void*)&gmap, (void*)&step0, (void*)&nchunk};
          err = b->adaptive ? hipLaunchCooperativeKernel(lrk::dp5_split_kernel(g.kp, g.nm != 0), dim3(g.wgs),
                                                         dim3(lrk::kTW), sargs_a, (unsigned)g.lds, gs)
                            : hipLaunchCooperativeKernel(lrk::packed_split_kernel(g.kp, g.nm != 0), dim3(g.wgs),
                                                         dim3(lrk::kTW), args, (unsigned)g.lds, gs);
        }
      } else if (g.packed) {
        const TrajDev* ptr = trajs + g.begin;
        if (b->adaptive) {
          const lrk::AdaptDev* aptr = ads + g.begin;
          void* pargs[] = {(void*)&ptr, (void*)&aptr, (void*)&step0, (void*)&nchunk};
          err = hipLaunchKernel(lrk::dp5_kernel(g.kp, prologue != 0, g.nm != 0), dim3(g.wgs), dim3(lrk::kTW), pargs,
                                g.lds, gs);
        } else {
          void* pargs[] = {(void*)&ptr, (void*)&step0, (void*)&nchunk};
          err = hipLaunchKernel(lrk::packed_kernel(g.kp, prologue != 0, g.nm != 0, g.gm, g.slots), dim3(g.wgs),
                                dim3(lrk::kTW), pargs, g.lds, gs);
        }
      } else {
        err = hipLaunchCooperativeKernel(persist_fn(g.rows, g.ge, g.prec, prologue != 0), dim3(g.wgs),
                                         dim3(lrk::kPW), args, (unsigned)g.lds, b->stream);
      }
      if (k >= 0) (void)hipEventRecord(b->ev[2 * k + 1], gs);
      return err == hipSuccess ? LR_OK : LR_ERR_HIP;
    };
    if (int e = launch(1, 0, 0)) return e;
    hipLaunchKernelGGL(lrk::k_obs, dim3(g.end - g.begin), dim3(lrk::kWG), 0, gs, trajs + g.begin,
                       (double*)nullptr);
    for (int64_t step = 0; step < g.max_steps;) {
      const int64_t chunk = std::min(g.chunk, g.max_steps - step);
      if (int e = launch(0, step, chunk)) return e;
      step += chunk;
      hipLaunchKernelGGL(lrk::k_obs, dim3(g.end - g.begin), dim3(lrk::kWG), 0, gs, trajs + g.begin,
                         (double*)nullptr);
    }
  }
  if (int e = join_all()) return e;
  for (int t = 0; t < b->n; ++t) {
    const TrajDev& v = b->dev[t];
    long long e = (long long)v.N * v.M;
    const int grid = (int)std::min<long long>((e + lrk::kWG - 1) / lrk::kWG, 4096);
    hipLaunchKernelGGL(lrk::k_to_abi, dim3(grid), dim3(lrk::kWG), 0, b->stream, trajs, t, v.Bb,
                       reinterpret_cast<double2*>(b->tr[t].d_B));
  }
  return hipGetLastError() == hipSuccess ? LR_OK : LR_ERR_HIP;
}
}  // namespace

extern "C" {

int lr_batch_status(lr_batch_t* b, int32_t* codes, int64_t* failed_steps) {
  if (!b) return LR_ERR_ARG;
  if (!b->ws) return LR_ERR_STATE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LR_ERR_HIP;
  int first = LR_OK;
  for (int i = 0; i < b->n; ++i) {
    const TrajDev& v = b->dev[b->pos[i]];
    int32_t st = 0;
    int64_t fs = -1;
    if (hipMemcpy(&st, v.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return LR_ERR_HIP;
    if (hipMemcpy(&fs, v.fail_step, sizeof(fs), hipMemcpyDeviceToHost) != hipSuccess) return LR_ERR_HIP;
    if (codes) codes[i] = st;
    if (failed_steps) failed_steps[i] = fs;
    if (first == LR_OK && st != LR_OK) first = st;
  }
  return first;
}

int lr_batch_profile_enable(lr_batch_t* b, int32_t on) {
  if (!b) return LR_ERR_ARG;
  b->prof = on != 0;
  b->n_ev = 0;
  return LR_OK;
}

int lr_batch_wait_limits(lr_batch_t* b, uint32_t spins, int32_t never) {
  if (!b) return LR_ERR_ARG;
  if (!b->ws) return LR_ERR_STATE;
  for (TrajDev& v : b->dev) {
    v.spin_limit = spins;
    v.wait_bias = never ? 1u : 0u;
  }
  const hipError_t e = hipMemcpyAsync(b->ws + b->off_trajs, b->dev.data(), sizeof(TrajDev) * (size_t)b->n,
                                      hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return LR_ERR_HIP;
  return hipStreamSynchronize(b->stream) == hipSuccess ? LR_OK : LR_ERR_HIP;
}

int lr_batch_profile_read(lr_batch_t* b, double* ms, int64_t* launches) {
  if (!b) return LR_ERR_ARG;
  if (b->stream && hipStreamSynchronize(b->stream) != hipSuccess) return LR_ERR_HIP;
  if (!b->stream && hipDeviceSynchronize() != hipSuccess) return LR_ERR_HIP;
  double tot = 0.0;
  for (int64_t k = 0; k < b->n_ev; ++k) {
    float x = 0.0f;
    if (hipEventElapsedTime(&x, b->ev[2 * k], b->ev[2 * k + 1]) == hipSuccess) tot += x;
  }
  if (ms) *ms = tot;
  if (launches) *launches = b->n_ev;
  return LR_OK;
}

void lr_batch_destroy(lr_batch_t* b) {
  if (!b) return;
  drop_graph(b);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->aux_ev) (void)hipEventDestroy(e);
  for (hipStream_t sx : b->aux) (void)hipStreamDestroy(sx);
  delete b;
}

}  // extern "C"
