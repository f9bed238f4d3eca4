// Operator application Z = H_eff(t) B on its own (the -i H_eff B term of the
// right-hand side of eq. "nosse", supplement S1.A), for any number of columns.
//
// The integrators fuse this stencil into their stage kernels; this kernel is
// the same operation as a stand-alone streaming pass over the caller's
// column-major layout, so that its memory bound can be measured (and used)
// by itself: every column of B is read once and every column of Z written
// once.  Columns are independent, so the factors of many trajectories of one
// model at one time can be applied in one launch side by side (ncols = K M).
//
// A workgroup takes one column at a time: the column (N complex entries,
// coalesced 16-byte loads) goes into LDS, then every thread forms its rows of
// Z from LDS -- the diagonal of H_eff, the couplings g (b+b^)(a+a^) and
// G (a+a^)(f+f^) (four taps each) and the drive d(t) (f+f^) (two taps), in
// the lab frame or the frame rotating at the carrier -- and writes them
// coalesced.  The workgroups stride over the columns; the loads of a
// workgroup's next column (up to kApPf entries per thread) are in flight in
// registers while it forms the current one, and both streams bypass the
// caches' retention (non-temporal: every byte is touched once).  Basis index
// n = (q d_r + r) d_f + f: filter neighbours are n +- 1, resonator n +- d_f,
// transmon n +- d_r d_f.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

constexpr int kApWG = 1024;    // threads of a workgroup (measured: 5.1 TB/s at N = 2000 against 4.2 with 256)
constexpr int kApMaxN = 8192;  // a column in LDS (128 KiB)
constexpr int kApPf = 2;       // entries per thread of the next column held in registers (N <= 2048 whole)

struct ApplyDev {
  int d_q, d_r, d_f, N;
  double w_q, alpha, w_r, w_f, g, G, kappa, gamma;
  double drv;      // d(t)
  double2 e1, e2;  // e^{i w_d t}, e^{2 i w_d t} (drive frame)
};

typedef double ap_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ap_load(const double2* p) {
  const ap_d2 v = __builtin_nontemporal_load(reinterpret_cast<const ap_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void ap_store(double2* p, double2 v) {
  ap_d2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<ap_d2*>(p));
}

template <bool ROT>
__global__ __launch_bounds__(kApWG) void k_apply_heff(ApplyDev D, const double2* __restrict__ B,
                                                      double2* __restrict__ Z, int64_t ncols) {
  extern __shared__ double2 col[];  // the column (N entries), then sqrt(0 .. dmax)
  const int N = D.N, d_q = D.d_q, d_r = D.d_r, d_f = D.d_f, tid = threadIdx.x;
  double* sqt = reinterpret_cast<double*>(col + N);
  const int dmax = max(max(d_q, d_r), d_f);
  for (int k = tid; k <= dmax; k += kApWG) sqt[k] = sqrt((double)k);
  const int sq_ = d_r * d_f;  // transmon stride
  const double2 e1 = D.e1, e2 = D.e2;
  const double2 e1c = make_double2(e1.x, -e1.y), e2c = make_double2(e2.x, -e2.y);
  double2 pf[kApPf];
  auto fetch = [&](int64_t c) {
    const double2* src = B + (size_t)c * N;
#pragma unroll
    for (int u = 0; u < kApPf; ++u) {
      const int n = tid + u * kApWG;
      if (n < N) pf[u] = ap_load(src + n);
    }
  };
  int64_t c = blockIdx.x;
  if (c < ncols) fetch(c);
  for (; c < ncols; c += gridDim.x) {
    __syncthreads();  // the previous column is consumed
#pragma unroll
    for (int u = 0; u < kApPf; ++u) {
      const int n = tid + u * kApWG;
      if (n < N) col[n] = pf[u];
    }
    for (int n = tid + kApPf * kApWG; n < N; n += kApWG) col[n] = ap_load(B + (size_t)c * N + n);
    __syncthreads();
    if (c + gridDim.x < ncols) fetch(c + gridDim.x);  // in flight while this column is formed
    double2* dst = Z + (size_t)c * N;
    for (int n = tid; n < N; n += kApWG) {
      const int q = n / sq_, rem = n - q * sq_, r = rem / d_f, f = rem - r * d_f;
      const double2 b = col[n];
      const double hr = D.w_q * q + 0.5 * D.alpha * q * (q - 1) + D.w_r * r + D.w_f * f;
      const double hi = -0.5 * (D.kappa * f + D.gamma * q);
      double2 z = make_double2(hr * b.x - hi * b.y, hr * b.y + hi * b.x);
      // c nb, with the phase ph in the rotating frame (real coefficient in the lab frame)
      auto tap = [&](double cf, double2 ph, const double2 nb) {
        if constexpr (ROT) {
          const double2 w = make_double2(cf * ph.x, cf * ph.y);
          z.x = fma(w.x, nb.x, z.x);
          z.x = fma(-w.y, nb.y, z.x);
          z.y = fma(w.x, nb.y, z.y);
          z.y = fma(w.y, nb.x, z.y);
        } else {
          z.x = fma(cf, nb.x, z.x);
          z.y = fma(cf, nb.y, z.y);
        }
      };
      const double2 ph0 = make_double2(1.0, 0.0);
      const double sq0 = sqt[q], sq1 = sqt[q + 1], sr0 = sqt[r], sr1 = sqt[r + 1], sf0 = sqt[f], sf1 = sqt[f + 1];
      // g (b + b^)(a + a^): (q -> q -+ 1) x (r -> r -+ 1); in the drive frame b^a^ (both raise,
      // neighbour with two fewer excitations) carries e^{2 i w_d t}, b a its conjugate
      if (q > 0) {
        if (r > 0) tap(D.g * sq0 * sr0, e2, col[n - sq_ - d_f]);
        if (r + 1 < d_r) tap(D.g * sq0 * sr1, ph0, col[n - sq_ + d_f]);
      }
      if (q + 1 < d_q) {
        if (r > 0) tap(D.g * sq1 * sr0, ph0, col[n + sq_ - d_f]);
        if (r + 1 < d_r) tap(D.g * sq1 * sr1, e2c, col[n + sq_ + d_f]);
      }
      // G (a + a^)(f + f^)
      if (f > 0) {
        if (r > 0) tap(D.G * sf0 * sr0, e2, col[n - d_f - 1]);
        if (r + 1 < d_r) tap(D.G * sf0 * sr1, ph0, col[n + d_f - 1]);
        tap(D.drv * sf0, e1, col[n - 1]);  // d(t) f^ (e^{i w_d t} in the drive frame)
      }
      if (f + 1 < d_f) {
        if (r > 0) tap(D.G * sf1 * sr0, ph0, col[n - d_f + 1]);
        if (r + 1 < d_r) tap(D.G * sf1 * sr1, e2c, col[n + d_f + 1]);
        tap(D.drv * sf1, e1c, col[n + 1]);  // d(t) f
      }
      ap_store(dst + n, z);
    }
  }
}

// Dynamic LDS bytes of k_apply_heff.
inline size_t apply_lds_bytes(int N, int dmax) { return (size_t)N * 16 + (size_t)(dmax + 2) * 8; }

}  // namespace lrk
