// Device-side descriptors and small helpers shared by the HIP kernels.
//
// Internal state layout ("layer-major"): row index
//     rho = (i_r * d_q + i_q) * d_f + i_f,   element (rho, j) at rho * M + j,
// interleaved complex.  One resonator layer (all i_q, i_f for a fixed i_r) is
// the contiguous block of L * M elements, L = d_q * d_f.  The jump operators
// (f on the filter, b on the transmon) never leave a layer, so Gram and cross
// products of a run of whole layers need no neighbours; only the resonator
// quadrature (a + a^) couples a layer to the layers above and below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrk {

constexpr int kWG = 256;          // threads per workgroup of the streaming kernels
constexpr int kMaxM = 32;         // largest supported rank
constexpr int kMaxPulseH = 63;    // heights of the smoothed stepwise envelope (n = nh + 1 <= 64 steps)
constexpr int kMaxDq = 8;         // transmon levels of the eigenbasis model (keeps TrajDev a small kernel argument)
constexpr int kMaxTileElems = 2048;  // rows*M of one tile (LDS budget: 32 KB of FP64 complex)
constexpr int kMaxElemsPerThread = kMaxTileElems / kWG;

enum Mode : int { MODE_STEP = 0, MODE_RHS = 1, MODE_GRAM = 2 };

struct TrajDev {
  // shape
  int32_t d_q, d_r, d_f, M;
  int32_t N, L, ntiles, obs_stride;
  int64_t nsteps;
  int64_t step_base;  // global index of step 0 of this call (stage times t0 + (step_base + n) dt)
  // model (rad/ns)
  double w_q, alpha, w_r, w_f, g, G, kappa, gamma;
  // drive
  int32_t pkind, prec;  // drive kind; arithmetic of the operator/Gram products (LR_FP64/FP32/BF16X3)
  int32_t frame, mkind; // 0 lab frame, 1 frame rotating at w_d (w_q, w_r, w_f then hold w - w_d); model kind
  double w_d, amp, t_ramp, T, p[6];
  int32_t nh, pad3;     // smoothed stepwise envelope: heights h_2 .. h_{nh+1}, logistic steepness
  double sigma, h[2 * kMaxPulseH];
  // time grid
  double t0, dt;
  // device buffers, internal layout
  double2* Bb;     // base state B_n (overwritten by B_{n+1} at the last stage)
  double2* S0;     // stage inputs (ping-pong)
  double2* S1;
  double2* acc;    // k1 + 2 k2 + 2 k3
  double2* W;      // [2 parity][2 jump][M*M]  W_k = (G^-1 C_k)^
  double2* part;   // [ntiles][3][M*M] Gram / cross-product partials per tile
  double* obs;     // caller's observation records (may be null)
  double* fro2;    // ||B^B||_F^2 of the last reduced Gram
  int64_t* step;   // device step counter
  int32_t* status; // first device error (0 = none)
  int64_t* fail_step;
  // persistent (on-chip) path: P workgroups of rt layers each
  int32_t P, rt;
  int32_t npe, pad1;    // entries of one Gram/cross partial (3 M^2)
  double2* SP;          // [2 parity][N*M] published stage states (tile boundary layers)
  double2* PART;        // [2 parity][P][npe] per-workgroup partials
  double2* RED;         // [2 parity][npe] reduced G, C_1, C_2
  uint32_t* flagA;      // [P * kFlagStride] "partials of stage g published" = g + 1
  uint32_t* flagB;      // [P * kFlagStride] "reduction of stage g done"     = g + 1
  uint32_t* abort_flag; // set when a bounded wait expires
  // model kinds 1, 2 (transmon eigenbasis): levels and charge operator (row-major d_q x d_q)
  double Et[kMaxDq];
  double ntq[kMaxDq * kMaxDq];
  // model kind 2 (normal-mode basis): s_21 .. s_24 of the filter operator, mu_l, mu_u, nu_l, nu_u
  double nm[8];
  // bounded waits of the group barriers: polls before a wait expires (0: kSpinLimit), and an offset
  // added to every barrier target (nonzero only to make every wait expire, for failure-handling tests)
  uint32_t spin_limit, wait_bias;
};

constexpr int kFlagStride = 32;    // one 128-byte line per flag

// Global-address-space views of descriptor pointers: loads and stores through
// them compile to global_* instead of flat_* instructions (flat accesses also
// count against the LDS wait counter and would serialise LDS traffic behind
// global memory latency).
typedef __attribute__((address_space(1))) double2 g_double2;
typedef __attribute__((address_space(1))) double g_double;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(1))) int64_t g_i64;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) {
  return make_double2(s * a.x, s * a.y);
}
__device__ __forceinline__ double2 cfma(double s, double2 a, double2 acc) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}
// acc + a * b and acc + conj(a) * b as four fused multiply-adds
__device__ __forceinline__ double2 cmac(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 cjmac(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}

// Cosine ramp r(x) of the flat-top window.
__host__ __device__ __forceinline__ double ramp_up(double x, double t_r) {
  if (x < 0.0) return 0.0;
  if (x >= t_r) return 1.0;
  return 0.5 * (1.0 - cos(M_PI * x / t_r));
}

// Drive coefficient d(t) multiplying (f + f^).
// e^{i w t} (the phase of a tap in the frame rotating at the drive carrier).
__host__ __device__ __forceinline__ double2 frame_phase(double w, double t) {
  return make_double2(cos(w * t), sin(w * t));
}

// Term j (1 <= j <= n = nh + 1) of the smoothed stepwise envelope:
// (h_{j+1} - h_j) f(t, j T / n, sigma), f the logistic function, h_1 = h_{n+1} = 0.
__host__ __device__ __forceinline__ double2 stepwise_term(const TrajDev& T, int j, double t) {
  const int n = T.nh + 1;
  const double2 hp = j <= T.nh ? make_double2(T.h[2 * (j - 1)], T.h[2 * (j - 1) + 1]) : make_double2(0.0, 0.0);
  const double2 hm = j >= 2 ? make_double2(T.h[2 * (j - 2)], T.h[2 * (j - 2) + 1]) : make_double2(0.0, 0.0);
  const double f = 1.0 / (1.0 + exp(-(t - j * T.T / n) / T.sigma));
  return make_double2((hp.x - hm.x) * f, (hp.y - hm.y) * f);
}

// Omega(t) of the smoothed stepwise envelope, steps summed in order (kept
// out of line: it runs once per stage time, away from the kernels' hot loops).
__host__ __device__ __attribute__((noinline)) inline double2 stepwise_envelope(const TrajDev& T, double t) {
  double2 om = make_double2(0.0, 0.0);
  for (int j = 1; j <= T.nh + 1; ++j) {
    const double2 v = stepwise_term(T, j, t);
    om.x += v.x;
    om.y += v.y;
  }
  return om;
}

// Drive coefficient d(t) on (f + f^).
__host__ __device__ __forceinline__ double drive_at(const TrajDev& T, double t) {
  if (T.pkind == 2) {  // Re[Omega(t) e^{-i w_d t}]
    const double2 om = stepwise_envelope(T, t);
    return om.x * cos(T.w_d * t) + om.y * sin(T.w_d * t);
  }
  if (T.pkind == 0) {
    return T.amp * ramp_up(t, T.t_ramp) * ramp_up(T.T - t, T.t_ramp) * cos(T.w_d * t);
  }
  const double a = 0.5 * T.T - 0.5 * T.t_ramp;
  double c;
  if (t <= a) c = 0.0;
  else if (t >= a + T.t_ramp) c = 1.0;
  else c = 0.5 * (1.0 - cos(M_PI * (t - a) / T.t_ramp));
  const double w1 = ramp_up(t, T.t_ramp) * (1.0 - c);
  const double w2 = ramp_up(T.T - t, T.t_ramp) * c;
  return T.p[0] * w1 * cos((T.w_d + T.p[2]) * t + T.p[1]) +
         T.p[3] * w2 * cos((T.w_d + T.p[5]) * t + T.p[4]);
}

}  // namespace lrk
