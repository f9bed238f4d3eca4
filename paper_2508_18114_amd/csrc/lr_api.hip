// Host side of the C ABI declared in include/lr.h: argument validation,
// workspace layout and the launch sequence of one RK4 integration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lr.h"
#include "lr_kernels.hip"
#include "lr_persistent.hip"
#include "lr_loss.hip"
#include "lr_dense.hip"
#include "lr_spectrum.hip"
#include "lr_packed.hip"
#include "lr_adaptive.hip"
#include "lr_apply.hip"

using lrk::TrajDev;

struct lr_ctx {
  lr_model_t model;
  int M = 0, prec = 0;
  int N = 0, L = 0, rt = 1, ntiles = 0;
  size_t off_traj = 0, off_tilemap = 0, off_rt = 0, off_Bb = 0, off_S0 = 0, off_S1 = 0, off_acc = 0,
         off_W = 0, off_part = 0, off_misc = 0, total = 0;
  // persistent path: P workgroups of prt layers
  int P = 0, prt = 1, prows = 2;
  size_t pers_lds = 0;
  size_t off_ptilemap = 0, off_SP = 0, off_PART = 0, off_RED = 0, off_flagA = 0, off_flagB = 0;
  bool persist_only = false;  // no multi-kernel buffers in the layout
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  TrajDev base{};
  // kernel timing telemetry
  bool prof = false;
  std::vector<hipEvent_t> ev_stage, ev_solve;  // start/stop pairs
  int64_t n_stage = 0, n_solve = 0;
};

// Workspace of lr_integrate_noalloc: a fixed array in device memory, one copy
// per GPU (each holds it until the process ends).  Host code never uses the
// array's name as an address: the device address of each GPU's copy comes
// from hipGetSymbolAddress on that device (scratch_ptr).
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace lrk {
// Device status of a trajectory (code, failing step) into caller memory.
__global__ void k_copy_status(const TrajDev* __restrict__ T, int64_t* dst) {
  dst[0] = *T->status;
  dst[1] = *T->fail_step;
}
// Tile map of the persistent kernel of one trajectory: workgroup w -> (0, w).
__global__ void k_fill_tilemap(int2* map, int P) {
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < P; w += gridDim.x * blockDim.x) map[w] = make_int2(0, w);
}
}  // namespace lrk

namespace {

constexpr double kDriveBound = 2.0 * M_PI * 0.4;  // |amplitude| < 2 pi 400 MHz
static_assert(lrk::kMaxPulseH == LR_PULSE_MAX_H, "stepwise heights of the device descriptor");
static_assert(lrk::kTMaxLM == LR_PACKED_MAX_LM, "layer size of the packed kernel");
static_assert(lrk::kMaxDq == LR_MAX_DQ, "transmon levels of the eigenbasis model");

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int check_pulse(const lr_pulse_t* p) {
  if (!p) return LR_ERR_ARG;
  if (p->kind != LR_PULSE_FLATTOP && p->kind != LR_PULSE_PIECEWISE6 && p->kind != LR_PULSE_STEPWISE)
    return LR_ERR_PULSE;
  if (p->frame != LR_FRAME_LAB && p->frame != LR_FRAME_DRIVE) return LR_ERR_PULSE;
  if (!(std::isfinite(p->w_d) && std::isfinite(p->T) && std::isfinite(p->t_ramp)) || p->t_ramp < 0.0)
    return LR_ERR_PULSE;
  if (p->kind == LR_PULSE_FLATTOP) {
    if (!(std::fabs(p->amp) < kDriveBound)) return LR_ERR_PULSE;
  } else if (p->kind == LR_PULSE_STEPWISE) {
    if (p->nh < 1 || p->nh > LR_PULSE_MAX_H || !(p->sigma > 0.0) || !std::isfinite(p->sigma) || !(p->T > 0.0))
      return LR_ERR_PULSE;
    for (int k = 0; k < p->nh; ++k)
      if (!(std::hypot(p->h[2 * k], p->h[2 * k + 1]) < kDriveBound)) return LR_ERR_PULSE;
  } else {
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(p->p[i])) return LR_ERR_PULSE;
    if (!(std::fabs(p->p[0]) < kDriveBound) || !(std::fabs(p->p[3]) < kDriveBound)) return LR_ERR_PULSE;
  }
  return LR_OK;
}

// Drive fields of a descriptor whose model fields are set; in the drive frame
// the mode frequencies become w - w_d (the frame change of the diagonal).
void set_pulse(TrajDev& v, const lr_pulse_t* p) {
  v.pkind = p->kind;
  v.frame = p->frame;
  if (p->frame == LR_FRAME_DRIVE) {
    v.w_q -= p->w_d;
    v.w_r -= p->w_d;
    v.w_f -= p->w_d;
  }
  v.w_d = p->w_d;
  v.amp = p->amp;
  v.t_ramp = p->t_ramp;
  v.T = p->T;
  for (int i = 0; i < 6; ++i) v.p[i] = p->p[i];
  v.nh = p->kind == LR_PULSE_STEPWISE ? p->nh : 0;
  v.sigma = p->sigma;
  for (int i = 0; i < 2 * LR_PULSE_MAX_H; ++i) v.h[i] = i < 2 * v.nh ? p->h[i] : 0.0;
}

TrajDev* dev_traj(const lr_ctx* c) { return reinterpret_cast<TrajDev*>(c->ws + c->off_traj); }
int2* dev_tilemap(const lr_ctx* c) { return reinterpret_cast<int2*>(c->ws + c->off_tilemap); }
int* dev_rt(const lr_ctx* c) { return reinterpret_cast<int*>(c->ws + c->off_rt); }

size_t stage_lds_bytes(const lr_ctx* c) {
  return (size_t)(2 * c->M * c->M + c->rt * c->L * c->M) * sizeof(double2);
}

int launch_ok() { return hipGetLastError() == hipSuccess ? LR_OK : LR_ERR_HIP; }

// Event pair slot for the next timed launch, or -1.
int prof_slot(lr_ctx* c, std::vector<hipEvent_t>& ev, int64_t& n) {
  if (!c->prof || n >= LR_PROFILE_MAX) return -1;
  const size_t need = 2 * (size_t)(n + 1);
  while (ev.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ev.push_back(e);
  }
  return (int)(n++);
}

void launch_stage(lr_ctx* c, int s, int mode) {
  const int k = prof_slot(c, c->ev_stage, c->n_stage);
  if (k >= 0) (void)hipEventRecord(c->ev_stage[2 * k], c->stream);
  hipLaunchKernelGGL(lrk::k_stage, dim3(c->ntiles), dim3(lrk::kWG), stage_lds_bytes(c), c->stream, dev_traj(c),
                     dev_tilemap(c), dev_rt(c), s, mode);
  if (k >= 0) (void)hipEventRecord(c->ev_stage[2 * k + 1], c->stream);
}

void launch_solve(lr_ctx* c, int wpar, int advance, int mode) {
  const int k = prof_slot(c, c->ev_solve, c->n_solve);
  if (k >= 0) (void)hipEventRecord(c->ev_solve[2 * k], c->stream);
  hipLaunchKernelGGL(lrk::k_solve, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), wpar, advance, mode);
  if (k >= 0) (void)hipEventRecord(c->ev_solve[2 * k + 1], c->stream);
}

int launch_persist(lr_ctx* c, int prologue, int64_t step0, int64_t nchunk) {
  const int k = prologue ? -1 : prof_slot(c, c->ev_stage, c->n_stage);
  if (k >= 0) (void)hipEventRecord(c->ev_stage[2 * k], c->stream);
  const TrajDev* tr = dev_traj(c);
  const int2* tmap = reinterpret_cast<const int2*>(c->ws + c->off_ptilemap);
  void* args[] = {(void*)&tr, (void*)&tmap, (void*)&step0, (void*)&nchunk};
  const void* fn = lrk::persist_kernel(c->prows, lrk::persist_ge(c->M), prologue != 0, c->prec);
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c->P), dim3(lrk::kPW), args, (unsigned)c->pers_lds, c->stream);
  if (k >= 0) (void)hipEventRecord(c->ev_stage[2 * k + 1], c->stream);
  return e == hipSuccess ? LR_OK : LR_ERR_HIP;
}

double prof_sum(const std::vector<hipEvent_t>& ev, int64_t n) {
  double tot = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess) tot += ms;
  }
  return tot;
}

int grid_for(const lr_ctx* c) {
  const long long e = (long long)c->N * c->M;
  long long g = (e + lrk::kWG - 1) / lrk::kWG;
  if (g > 4096) g = 4096;
  return (int)g;
}

// Enqueue: descriptor, reset, B -> internal, Gram of B, solve (W for stage 0).
int prologue(lr_ctx* c, const TrajDev& v, const lr_c64* d_B) {
  hipLaunchKernelGGL(lrk::k_set_traj, dim3(1), dim3(1), 0, c->stream, dev_traj(c), v);
  hipLaunchKernelGGL(lrk::k_reset, dim3(1), dim3(64), 0, c->stream, dev_traj(c), 1);
  hipLaunchKernelGGL(lrk::k_to_internal, dim3(grid_for(c)), dim3(lrk::kWG), 0, c->stream, dev_traj(c), 0,
                     reinterpret_cast<const double2*>(d_B), c->base.Bb);
  launch_stage(c, 0, lrk::MODE_GRAM);
  return launch_ok();
}

// Validation and workspace layout of a context (lr_init); persist_only leaves
// out the buffers of the multi-kernel path.
int ctx_setup(lr_ctx* c, const lr_model_t* m, int32_t M, int32_t precision, bool persist_only) {
  if (m->kind != LR_MODEL_DUFFING) return LR_ERR_ARG;  // the eigenbasis model runs in packed batches only
  if (m->d_q < 2 || m->d_r < 1 || m->d_f < 1) return LR_ERR_ARG;
  const long long N = (long long)m->d_q * m->d_r * m->d_f;
  if (N > (1LL << 26)) return LR_ERR_ARG;
  if (M < 1 || M > LR_MAX_M || M > N) return LR_ERR_ARG;
  if (precision != LR_FP64 && precision != LR_FP32 && precision != LR_BF16X3) return LR_ERR_ARG;
  const double vals[] = {m->w_q, m->alpha, m->w_r, m->w_f, m->g, m->G, m->kappa_f, m->gamma_1};
  for (double x : vals)
    if (!std::isfinite(x)) return LR_ERR_ARG;
  if (m->kappa_f < 0.0 || m->gamma_1 < 0.0) return LR_ERR_ARG;
  const int L = m->d_q * m->d_f;
  if ((long long)L * M > lrk::kMaxTileElems) return LR_ERR_ARG;

  c->model = *m;
  c->M = M;
  c->prec = precision;
  c->N = (int)N;
  c->L = L;
  int rt = 1;
  if (const char* e = std::getenv("LR_TILE_LAYERS")) rt = std::atoi(e);
  const int rt_max = lrk::kMaxTileElems / (L * M);
  if (rt < 1) rt = 1;
  if (rt > rt_max) rt = rt_max;
  if (rt > m->d_r) rt = m->d_r;
  c->rt = rt;
  c->ntiles = (m->d_r + rt - 1) / rt;

  // persistent path: smallest layer count per workgroup that fits the
  // register rows (<= kMaxRowsPerThread per thread) and the 160 KB LDS
  {
    int prt = 1;
    if (const char* e = std::getenv("LR_PERSIST_LAYERS")) prt = std::atoi(e);
    if (prt < 1) prt = 1;
    if (prt > m->d_r) prt = m->d_r;
    const int NG = lrk::kPW / M;
    while (prt > 1 && ((prt * L + NG - 1) / NG > lrk::kMaxRowsPerThread || lrk::persist_lds_bytes(prt, L, M, (m->d_r + prt - 1) / prt) > lrk::kPersistLdsMax))
      --prt;
    c->prt = prt;
    c->prows = ((prt * L + NG - 1) / NG <= 2) ? 2 : 3;
    c->P = (m->d_r + prt - 1) / prt;
    c->pers_lds = lrk::persist_lds_bytes(prt, L, M, c->P);
    if ((L + NG - 1) / NG > lrk::kMaxRowsPerThread || c->pers_lds > lrk::kPersistLdsMax) c->P = 0;  // path unavailable
  }
  const size_t a = 256, nm = (size_t)N * M * sizeof(double2), mm = (size_t)M * M * sizeof(double2);
  size_t o = 0;
  c->persist_only = persist_only;
  c->off_traj = o;    o = align_up(o + sizeof(TrajDev), a);
  c->off_Bb = o;      o = align_up(o + nm, a);
  c->off_misc = o;    o = align_up(o + 64, a);
  if (!persist_only) {  // the multi-kernel path (lr_rhs, lr_observables, fallback)
    c->off_tilemap = o; o = align_up(o + (size_t)c->ntiles * sizeof(int2), a);
    c->off_rt = o;      o = align_up(o + sizeof(int), a);
    c->off_S0 = o;      o = align_up(o + nm, a);
    c->off_S1 = o;      o = align_up(o + nm, a);
    c->off_acc = o;     o = align_up(o + nm, a);
    c->off_W = o;       o = align_up(o + 4 * mm, a);
    c->off_part = o;    o = align_up(o + (size_t)c->ntiles * 3 * mm, a);
  }
  if (c->P > 0) {
    const size_t npe = 3 * mm;
    c->off_ptilemap = o; o = align_up(o + (size_t)c->P * sizeof(int2), a);
    c->off_SP = o;       o = align_up(o + 2 * nm, a);
    c->off_PART = o;     o = align_up(o + 2 * (size_t)c->P * npe, a);
    c->off_RED = o;      o = align_up(o + 2 * npe, a);
    c->off_flagA = o;    o = align_up(o + (size_t)c->P * lrk::kFlagStride * 4, a);
    c->off_flagB = o;    o = align_up(o + (size_t)c->P * lrk::kFlagStride * 4, a);
  }
  c->total = o;

  TrajDev& b = c->base;
  b.d_q = m->d_q; b.d_r = m->d_r; b.d_f = m->d_f; b.M = M;
  b.N = (int)N; b.L = L; b.ntiles = c->ntiles; b.obs_stride = 0;
  b.nsteps = 0;
  b.w_q = m->w_q; b.alpha = m->alpha; b.w_r = m->w_r; b.w_f = m->w_f;
  b.g = m->g; b.G = m->G; b.kappa = m->kappa_f; b.gamma = m->gamma_1;
  return LR_OK;
}


// Device pointers of a context's descriptor into the workspace ws.
void ctx_pointers(lr_ctx* c, char* ws, hipStream_t stream) {
  c->ws = ws;
  c->stream = stream;
  TrajDev& b = c->base;
  auto at = [&](size_t off) { return reinterpret_cast<double2*>(c->ws + off); };
  b.Bb = at(c->off_Bb);
  b.S0 = c->persist_only ? nullptr : at(c->off_S0);
  b.S1 = c->persist_only ? nullptr : at(c->off_S1);
  b.acc = c->persist_only ? nullptr : at(c->off_acc);
  b.W = c->persist_only ? nullptr : at(c->off_W);
  b.part = c->persist_only ? nullptr : at(c->off_part);
  b.step = reinterpret_cast<int64_t*>(c->ws + c->off_misc);
  b.fail_step = reinterpret_cast<int64_t*>(c->ws + c->off_misc + 8);
  b.fro2 = reinterpret_cast<double*>(c->ws + c->off_misc + 16);
  b.status = reinterpret_cast<int32_t*>(c->ws + c->off_misc + 24);
  b.abort_flag = reinterpret_cast<uint32_t*>(c->ws + c->off_misc + 28);
  b.obs = nullptr;
  b.P = c->P;
  b.rt = c->prt;
  b.npe = 3 * c->M * c->M;
  b.prec = c->prec;
  if (c->P > 0) {
    b.SP = at(c->off_SP);
    b.PART = at(c->off_PART);
    b.RED = at(c->off_RED);
    b.flagA = reinterpret_cast<uint32_t*>(c->ws + c->off_flagA);
    b.flagB = reinterpret_cast<uint32_t*>(c->ws + c->off_flagB);
  }
}

// Enqueue the integration of descriptor v (pulse, times, records set) on the
// persistent on-chip path of a bound context: descriptor, resets, layout in,
// prologue, chunks of steps with records, layout out.
int integrate_persist(lr_ctx* c, const TrajDev& v, int64_t nsteps, lr_c64* d_B, int32_t obs_stride) {
  hipLaunchKernelGGL(lrk::k_set_traj, dim3(1), dim3(1), 0, c->stream, dev_traj(c), v);
  hipLaunchKernelGGL(lrk::k_reset, dim3(1), dim3(64), 0, c->stream, dev_traj(c), 1);
  hipLaunchKernelGGL(lrk::k_reset_persist, dim3(1), dim3(256), 0, c->stream, dev_traj(c), 1);
  hipLaunchKernelGGL(lrk::k_to_internal, dim3(grid_for(c)), dim3(lrk::kWG), 0, c->stream, dev_traj(c), 0,
                     reinterpret_cast<const double2*>(d_B), c->base.Bb);
  if (int e = launch_ok()) return e;
  if (int e = launch_persist(c, 1, 0, 0)) return e;
  if (obs_stride > 0)
    hipLaunchKernelGGL(lrk::k_obs, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), (double*)nullptr);
  const int64_t max_chunk = obs_stride > 0 ? obs_stride : 4096;
  for (int64_t step = 0; step < nsteps;) {
    const int64_t chunk = (nsteps - step < max_chunk) ? nsteps - step : max_chunk;
    if (int e = launch_persist(c, 0, step, chunk)) return e;
    step += chunk;
    if (obs_stride > 0 && step % obs_stride == 0)
      hipLaunchKernelGGL(lrk::k_obs, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), (double*)nullptr);
  }
  hipLaunchKernelGGL(lrk::k_to_abi, dim3(grid_for(c)), dim3(lrk::kWG), 0, c->stream, dev_traj(c), 0, c->base.Bb,
                     reinterpret_cast<double2*>(d_B));
  return launch_ok();
}

// Dynamic-LDS attribute of the persistent kernels of a context's variant.
int persist_attributes(const lr_ctx* c) {
  for (int pro = 0; pro < 2; ++pro) {
    const void* fn = lrk::persist_kernel(c->prows, lrk::persist_ge(c->M), pro != 0, c->prec);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->pers_lds) != hipSuccess)
      return LR_ERR_HIP;
  }
  return LR_OK;
}

// Device address of the current GPU's copy of `scratch` (looked up once per
// device, with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LR_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return LR_OK;
}

}  // namespace

extern "C" {

const char* lr_strerror(int code) {
  switch (code) {
    case LR_OK: return "ok";
    case LR_ERR_ARG: return "invalid argument";
    case LR_ERR_OOM: return "workspace too small";
    case LR_ERR_HIP: return "HIP runtime error";
    case LR_ERR_GRAM_NOT_PD: return "Gram matrix B^B not positive definite (elimination pivot <= 0)";
    case LR_ERR_NONFINITE: return "non-finite state";
    case LR_ERR_PULSE: return "invalid pulse (unknown kind or amplitude above 2*pi*0.4 rad/ns)";
    case LR_ERR_STATE: return "invalid call order (no workspace bound)";
    case LR_ERR_TIMEOUT: return "device-side wait expired";
    case LR_ERR_STEP: return "adaptive step size underflow or step budget spent";
    default: return "unknown error";
  }
}

int lr_init(lr_ctx_t** out, const lr_model_t* m, int32_t M, int32_t precision) {
  if (!out || !m) return LR_ERR_ARG;
  *out = nullptr;
  lr_ctx* c = new (std::nothrow) lr_ctx();
  if (!c) return LR_ERR_OOM;
  if (int e = ctx_setup(c, m, M, precision, false)) {
    delete c;
    return e;
  }
  *out = c;
  return LR_OK;
}

size_t lr_workspace_bytes(const lr_ctx_t* c) { return c ? c->total : 0; }

int lr_bind(lr_ctx_t* c, void* d_ws, size_t bytes, void* stream) {
  if (!c || !d_ws) return LR_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return LR_ERR_ARG;
  if (bytes < c->total) return LR_ERR_OOM;
  ctx_pointers(c, static_cast<char*>(d_ws), static_cast<hipStream_t>(stream));

  // static tile map of this shape (one entry per workgroup of k_stage)
  const int nmap = c->ntiles > c->P ? c->ntiles : c->P;
  int2* tm = new (std::nothrow) int2[nmap];
  if (!tm) return LR_ERR_OOM;
  for (int t = 0; t < nmap; ++t) tm[t] = make_int2(0, t);
  hipError_t e1 = hipMemcpyAsync(dev_tilemap(c), tm, sizeof(int2) * c->ntiles, hipMemcpyHostToDevice, c->stream);
  hipError_t e2 = hipMemcpyAsync(dev_rt(c), &c->rt, sizeof(int), hipMemcpyHostToDevice, c->stream);
  hipError_t e4 = hipSuccess;
  if (c->P > 0)
    e4 = hipMemcpyAsync(c->ws + c->off_ptilemap, tm, sizeof(int2) * c->P, hipMemcpyHostToDevice, c->stream);
  // a defined device status from the start (lr_status before any integration)
  hipLaunchKernelGGL(lrk::k_set_traj, dim3(1), dim3(1), 0, c->stream, dev_traj(c), c->base);
  hipLaunchKernelGGL(lrk::k_reset, dim3(1), dim3(64), 0, c->stream, dev_traj(c), 1);
  hipError_t e3 = hipStreamSynchronize(c->stream);
  delete[] tm;
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) return LR_ERR_HIP;
  if (c->P > 0) return persist_attributes(c);
  return LR_OK;
}

int lr_rhs(lr_ctx_t* c, const lr_pulse_t* pulse, double t, const lr_c64* d_B, lr_c64* d_dB) {
  if (!c || !d_B || !d_dB || !std::isfinite(t)) return LR_ERR_ARG;
  if (!c->ws) return LR_ERR_STATE;
  if (int e = check_pulse(pulse)) return e;
  TrajDev v = c->base;
  set_pulse(v, pulse);
  v.t0 = t;
  v.dt = 0.0;
  v.nsteps = 0;
  if (int e = prologue(c, v, d_B)) return e;
  launch_solve(c, 0, 0, lrk::MODE_RHS);
  launch_stage(c, 0, lrk::MODE_RHS);
  hipLaunchKernelGGL(lrk::k_to_abi, dim3(grid_for(c)), dim3(lrk::kWG), 0, c->stream, dev_traj(c), 0,
                     c->base.acc, reinterpret_cast<double2*>(d_dB));
  return launch_ok();
}

int lr_integrate(lr_ctx_t* c, const lr_pulse_t* pulse, double t0, double dt, int64_t nsteps, lr_c64* d_B,
                 int32_t obs_stride, double* d_obs) {
  if (!c || !d_B || !std::isfinite(t0) || !(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || obs_stride < 0)
    return LR_ERR_ARG;
  if (obs_stride > 0 && !d_obs) return LR_ERR_ARG;
  if (!c->ws) return LR_ERR_STATE;
  if (int e = check_pulse(pulse)) return e;
  TrajDev v = c->base;
  set_pulse(v, pulse);
  v.t0 = t0;
  v.dt = dt;
  v.nsteps = nsteps;
  v.obs = obs_stride > 0 ? d_obs : nullptr;
  v.obs_stride = obs_stride;
  // the reduced-precision modes exist on the persistent path only
  if (c->prec != LR_FP64 && (c->P == 0 || std::getenv("LR_NO_PERSIST"))) return LR_ERR_ARG;
  if (c->P > 0 && !std::getenv("LR_NO_PERSIST")) return integrate_persist(c, v, nsteps, d_B, obs_stride);
  if (int e = prologue(c, v, d_B)) return e;
  launch_solve(c, 0, 0, lrk::MODE_RHS);
  if (obs_stride > 0)
    hipLaunchKernelGGL(lrk::k_obs, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), (double*)nullptr);
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 4; ++s) {
      launch_stage(c, s, lrk::MODE_STEP);
      launch_solve(c, (s + 1) & 1, s == 3, lrk::MODE_STEP);
    }
    if (obs_stride > 0 && (n + 1) % obs_stride == 0)
      hipLaunchKernelGGL(lrk::k_obs, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), (double*)nullptr);
    if ((n & 1023) == 1023 && hipGetLastError() != hipSuccess) return LR_ERR_HIP;
  }
  hipLaunchKernelGGL(lrk::k_to_abi, dim3(grid_for(c)), dim3(lrk::kWG), 0, c->stream, dev_traj(c), 0,
                     c->base.Bb, reinterpret_cast<double2*>(d_B));
  return launch_ok();
}

int lr_observables(lr_ctx_t* c, const lr_c64* d_B, double* d_out) {
  if (!c || !d_B || !d_out) return LR_ERR_ARG;
  if (!c->ws) return LR_ERR_STATE;
  TrajDev v = c->base;
  v.pkind = 0;
  v.nsteps = 0;
  if (int e = prologue(c, v, d_B)) return e;
  launch_solve(c, 0, 0, lrk::MODE_GRAM);
  hipLaunchKernelGGL(lrk::k_obs, dim3(1), dim3(lrk::kWG), 0, c->stream, dev_traj(c), d_out);
  return launch_ok();
}

int lr_spectrum(lr_ctx_t* c, const lr_c64* d_B, double* d_eval) {
  if (!c || !d_B || !d_eval) return LR_ERR_ARG;
  if (!c->ws) return LR_ERR_STATE;
  hipLaunchKernelGGL(lrk::k_spectrum, dim3(1), dim3(lrk::kSpecWG), 0, c->stream,
                     reinterpret_cast<const double2*>(d_B), c->N, c->M, d_eval);
  return launch_ok();
}

int lr_status(lr_ctx_t* c, int64_t* failed_step) {
  if (!c) return LR_ERR_ARG;
  if (!c->ws) return LR_ERR_STATE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LR_ERR_HIP;
  int32_t st = 0;
  int64_t fs = -1;
  if (hipMemcpy(&st, c->base.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return LR_ERR_HIP;
  if (hipMemcpy(&fs, c->base.fail_step, sizeof(fs), hipMemcpyDeviceToHost) != hipSuccess) return LR_ERR_HIP;
  if (failed_step) *failed_step = fs;
  return st;
}

int lr_profile_enable(lr_ctx_t* c, int32_t on) {
  if (!c) return LR_ERR_ARG;
  c->prof = on != 0;
  c->n_stage = c->n_solve = 0;
  return LR_OK;
}

int lr_wait_limits(lr_ctx_t* c, uint32_t spins, int32_t never) {
  if (!c) return LR_ERR_ARG;
  c->base.spin_limit = spins;
  c->base.wait_bias = never ? 1u : 0u;
  return LR_OK;
}

int lr_profile_read(lr_ctx_t* c, double* stage_ms, int64_t* stage_launches, double* solve_ms,
                    int64_t* solve_launches) {
  if (!c) return LR_ERR_ARG;
  if (c->stream && hipStreamSynchronize(c->stream) != hipSuccess) return LR_ERR_HIP;
  if (!c->stream && hipDeviceSynchronize() != hipSuccess) return LR_ERR_HIP;
  if (stage_ms) *stage_ms = prof_sum(c->ev_stage, c->n_stage);
  if (stage_launches) *stage_launches = c->n_stage;
  if (solve_ms) *solve_ms = prof_sum(c->ev_solve, c->n_solve);
  if (solve_launches) *solve_launches = c->n_solve;
  return LR_OK;
}

int lr_readout_loss(const double* d_obs_g, const double* d_obs_e, int64_t nsamples, int32_t d_q, double h,
                    double kappa_f, double gamma_1, double eta, double* d_out, void* stream) {
  if (!d_obs_g || !d_obs_e || !d_out || nsamples < 2 || d_q < 2) return LR_ERR_ARG;
  if (!(std::isfinite(h) && h > 0.0 && std::isfinite(kappa_f) && kappa_f >= 0.0 && std::isfinite(gamma_1) &&
        gamma_1 >= 0.0 && std::isfinite(eta) && eta >= 0.0))
    return LR_ERR_ARG;
  hipLaunchKernelGGL(lrk::k_readout_loss, dim3(1), dim3(lrk::kLossWG), 0, (hipStream_t)stream, d_obs_g, d_obs_e,
                     nsamples, (int)LR_OBS_LEN(d_q), (int)d_q, h, kappa_f, gamma_1, eta, d_out);
  return hipGetLastError() == hipSuccess ? LR_OK : LR_ERR_HIP;
}

size_t lr_dense_workspace_bytes(const lr_model_t* m) {
  if (!m || m->d_q < 1 || m->d_r < 1 || m->d_f < 1) return 0;
  const size_t N = (size_t)m->d_q * m->d_r * m->d_f;
  return 4 * N * N * sizeof(double2);
}

int lr_dense_integrate(const lr_model_t* m, const lr_pulse_t* pulse, double t0, double dt, int64_t nsteps,
                       lr_c64* d_rho, int32_t obs_stride, double* d_obs, void* d_workspace, size_t bytes,
                       void* stream) {
  if (!m || !d_rho || !d_workspace || m->d_q < 1 || m->d_r < 1 || m->d_f < 1) return LR_ERR_ARG;
  if (m->kind != LR_MODEL_DUFFING) return LR_ERR_ARG;
  const long long Nl = (long long)m->d_q * m->d_r * m->d_f;
  if (Nl > 16384) return LR_ERR_ARG;
  if (bytes < lr_dense_workspace_bytes(m)) return LR_ERR_ARG;
  if (!(std::isfinite(dt) && dt > 0.0 && std::isfinite(t0)) || nsteps < 0) return LR_ERR_ARG;
  if (obs_stride < 0 || (obs_stride > 0 && !d_obs)) return LR_ERR_ARG;
  if (int e = check_pulse(pulse)) return e;
  const double vals[] = {m->w_q, m->alpha, m->w_r, m->w_f, m->g, m->G, m->kappa_f, m->gamma_1};
  for (double x : vals)
    if (!std::isfinite(x)) return LR_ERR_ARG;
  if (m->kappa_f < 0.0 || m->gamma_1 < 0.0) return LR_ERR_ARG;
  const int N = (int)Nl;
  TrajDev pv{};
  pv.w_q = m->w_q;
  pv.w_r = m->w_r;
  pv.w_f = m->w_f;
  set_pulse(pv, pulse);
  const bool rot = pulse->frame == LR_FRAME_DRIVE;
  lrk::DenseDev D{m->d_q, m->d_r, m->d_f, N, rot ? 1 : 0, pv.w_q, m->alpha, pv.w_r, pv.w_f, m->g, m->G, m->kappa_f,
                  m->gamma_1};
  hipStream_t st = (hipStream_t)stream;
  double2* base = reinterpret_cast<double2*>(d_rho);
  double2* X1 = reinterpret_cast<double2*>(d_workspace);
  double2* X2 = X1 + (size_t)N * N;
  double2* acc = X2 + (size_t)N * N;
  double2* Z = acc + (size_t)N * N;
  const dim3 ga((N + lrk::kDenseWG - 1) / lrk::kDenseWG, N), gc((N + 31) / 32, (N + 31) / 32);
  const int rec = 6 + m->d_q;
  if (obs_stride > 0) hipLaunchKernelGGL(lrk::k_dense_obs, dim3(1), dim3(lrk::kDenseWG), 0, st, D, base, d_obs);
  int64_t nrec = 1;
  for (int64_t n = 0; n < nsteps; ++n) {
    const double t = t0 + (double)n * dt;
    const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    const double2* in[4] = {base, X1, X2, X1};
    double2* out[4] = {X1, X2, X1, nullptr};
    for (int s = 0; s < 4; ++s) {
      const double ts = t + cs[s] * dt;
      const double drv = lrk::drive_at(pv, ts);
      const double2 e1 = lrk::frame_phase(pv.w_d, ts), e2 = lrk::frame_phase(2.0 * pv.w_d, ts);
      hipLaunchKernelGGL(lrk::k_dense_apply, ga, dim3(lrk::kDenseWG), 0, st, D, drv, e1, e2, in[s], Z);
      hipLaunchKernelGGL(lrk::k_dense_combine, gc, dim3(lrk::kDenseWG), 0, st, D, in[s], Z, base, acc, out[s], s,
                         dt);
    }
    if (obs_stride > 0 && (n + 1) % obs_stride == 0)
      hipLaunchKernelGGL(lrk::k_dense_obs, dim3(1), dim3(lrk::kDenseWG), 0, st, D, base, d_obs + (nrec++) * rec);
  }
  return hipGetLastError() == hipSuccess ? LR_OK : LR_ERR_HIP;
}

int lr_apply_heff(const lr_model_t* m, const lr_pulse_t* pulse, double t, const lr_c64* d_B, int64_t ncols,
                  lr_c64* d_Z, void* stream) {
  if (!m || !d_B || !d_Z || ncols < 0 || !std::isfinite(t)) return LR_ERR_ARG;
  if (m->kind != LR_MODEL_DUFFING || m->d_q < 1 || m->d_r < 1 || m->d_f < 1) return LR_ERR_ARG;
  const long long Nl = (long long)m->d_q * m->d_r * m->d_f;
  if (Nl > lrk::kApMaxN) return LR_ERR_ARG;
  const double vals[] = {m->w_q, m->alpha, m->w_r, m->w_f, m->g, m->G, m->kappa_f, m->gamma_1};
  for (double x : vals)
    if (!std::isfinite(x)) return LR_ERR_ARG;
  if (m->kappa_f < 0.0 || m->gamma_1 < 0.0) return LR_ERR_ARG;
  if (int e = check_pulse(pulse)) return e;
  if (reinterpret_cast<const char*>(d_B) < reinterpret_cast<const char*>(d_Z) + Nl * ncols * 16 &&
      reinterpret_cast<const char*>(d_Z) < reinterpret_cast<const char*>(d_B) + Nl * ncols * 16)
    return LR_ERR_ARG;  // B and Z overlap
  if (ncols == 0) return LR_OK;
  TrajDev pv{};
  pv.w_q = m->w_q;
  pv.w_r = m->w_r;
  pv.w_f = m->w_f;
  set_pulse(pv, pulse);
  const bool rot = pulse->frame == LR_FRAME_DRIVE;
  lrk::ApplyDev D{m->d_q, m->d_r, m->d_f, (int)Nl, pv.w_q, m->alpha, pv.w_r, pv.w_f, m->g, m->G, m->kappa_f,
                  m->gamma_1, lrk::drive_at(pv, t), lrk::frame_phase(pulse->w_d, t),
                  lrk::frame_phase(2.0 * pulse->w_d, t)};
  const int dmax = std::max(std::max(m->d_q, m->d_r), m->d_f);
  const size_t lds = lrk::apply_lds_bytes((int)Nl, dmax);
  const void* fn = rot ? (const void*)lrk::k_apply_heff<true> : (const void*)lrk::k_apply_heff<false>;
  if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return LR_ERR_HIP;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return LR_ERR_HIP;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, lrk::kApWG, lds) != hipSuccess || per_cu < 1)
    return LR_ERR_HIP;
  // two resident waves of workgroups, each striding over its columns with the next one in flight
  const long long grid = std::min<long long>(ncols, 2LL * per_cu * ncu);
  const double2* Bp = reinterpret_cast<const double2*>(d_B);
  double2* Zp = reinterpret_cast<double2*>(d_Z);
  if (rot)
    hipLaunchKernelGGL(lrk::k_apply_heff<true>, dim3((unsigned)grid), dim3(lrk::kApWG), lds, (hipStream_t)stream, D,
                       Bp, Zp, (int64_t)ncols);
  else
    hipLaunchKernelGGL(lrk::k_apply_heff<false>, dim3((unsigned)grid), dim3(lrk::kApWG), lds, (hipStream_t)stream, D,
                       Bp, Zp, (int64_t)ncols);
  return launch_ok();
}

int lr_integrate_noalloc(const lr_model_t* m, int32_t M, int32_t precision, const lr_pulse_t* pulse, double t0,
                         double dt, int64_t nsteps, lr_c64* d_B, int32_t obs_stride, double* d_obs,
                         int64_t* d_status, void* stream) {
  if (!m || !d_B || !std::isfinite(t0) || !(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || obs_stride < 0)
    return LR_ERR_ARG;
  if (obs_stride > 0 && !d_obs) return LR_ERR_ARG;
  if (int e = check_pulse(pulse)) return e;
  lr_ctx c;  // host descriptor on the stack: no allocation
  if (int e = ctx_setup(&c, m, M, precision, true)) return e;
  if (c.P == 0) return LR_ERR_ARG;                        // no persistent configuration for this shape
  if (c.total > kNoallocScratchBytes) return LR_ERR_OOM;  // above the fixed workspace
  char* ws = nullptr;
  if (int e = scratch_ptr(&ws)) return e;
  ctx_pointers(&c, ws, static_cast<hipStream_t>(stream));
  if (int e = persist_attributes(&c)) return e;
  hipLaunchKernelGGL(lrk::k_fill_tilemap, dim3(1), dim3(256), 0, c.stream,
                     reinterpret_cast<int2*>(c.ws + c.off_ptilemap), c.P);
  TrajDev v = c.base;
  set_pulse(v, pulse);
  v.t0 = t0;
  v.dt = dt;
  v.nsteps = nsteps;
  v.obs = obs_stride > 0 ? d_obs : nullptr;
  v.obs_stride = obs_stride;
  if (int e = integrate_persist(&c, v, nsteps, d_B, obs_stride)) return e;
  if (d_status)
    hipLaunchKernelGGL(lrk::k_copy_status, dim3(1), dim3(1), 0, c.stream, dev_traj(&c), d_status);
  return launch_ok();
}

void lr_destroy(lr_ctx_t* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev_stage) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_solve) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"

#include "lr_batch.hip"
