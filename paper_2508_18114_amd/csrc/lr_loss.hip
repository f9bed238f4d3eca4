// Readout figures of merit from the observation series of a g/e trajectory
// pair (Supplement S3.A, eqs. "SNR", "separation_error",
// "assignment_error"; S3.B, eqs. "transmon_ionization", "loss_function").
//
// One workgroup: every thread accumulates the composite-trapezoid sums of
// its samples (strided, in order), then a fixed-order tree over the
// workgroup; thread 0 forms the six outputs.
#include <hip/hip_runtime.h>

namespace lrk {

constexpr int kLossWG = 256;

__global__ __launch_bounds__(kLossWG) void k_readout_loss(const double* __restrict__ obs_g,
                                                           const double* __restrict__ obs_e, int64_t n, int ld,
                                                           int d_q, double h, double kappa_f, double gamma_1,
                                                           double eta, double* __restrict__ out) {
  __shared__ double s_sep[kLossWG];
  __shared__ double s_ion[kLossWG];
  double sep = 0.0, ion = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kLossWG) {
    const double w = (i == 0 || i == n - 1) ? 0.5 : 1.0;  // trapezoid weight (times h below)
    const double* g = obs_g + i * ld;
    const double* e = obs_e + i * ld;
    const double dr = e[2] - g[2], di = e[3] - g[3];  // beta_e - beta_g, beta = <f>
    sep += w * (dr * dr + di * di);
    double p = 0.0;
    for (int k = 2; k < d_q; ++k) p += g[6 + k] + e[6 + k];  // levels beyond g, e
    ion += w * p;
  }
  s_sep[threadIdx.x] = sep;
  s_ion[threadIdx.x] = ion;
  __syncthreads();
  for (int off = kLossWG / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_sep[threadIdx.x] += s_sep[threadIdx.x + off];
      s_ion[threadIdx.x] += s_ion[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tau = h * (double)(n - 1);
    const double snr = sqrt(2.0 * eta * kappa_f * h * s_sep[0]);
    const double eps_sep = 0.5 * erfc(0.5 * snr);
    const double eps_decay = 0.5 * tau * gamma_1;
    const double eps_a = eps_sep + eps_decay;
    const double ionisation = h * s_ion[0] / tau;
    out[0] = snr;
    out[1] = eps_sep;
    out[2] = eps_decay;
    out[3] = eps_a;
    out[4] = ionisation;
    out[5] = log10(eps_a + ionisation);
  }
}

}  // namespace lrk
