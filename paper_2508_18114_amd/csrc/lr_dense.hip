// Dense full-Lindblad RK4 integrator (the comparison solve of the low-rank
// method at the same N): the master equation of Supplement S1.A
// (eq. "master_equation" with the dissipator of eq. "lindblad_dissipator"),
//
//   d rho/dt = -i [H, rho] + sum_k ( L_k rho L_k^ - 1/2 {L_k^ L_k, rho} )
//            = Y + Y^ + sum_k L_k rho L_k^,     Y = -i H_eff rho,
//
// with H_eff = H - i/2 (kappa_f n_f + gamma_1 n_q), the same model and drive
// as the low-rank path, on a dense N x N rho in the ABI basis order
// n = (q d_r + r) d_f + f (row-major, interleaved complex FP64).
//
// Per RK4 stage two streaming kernels:
//   k_dense_apply    Z = -i H_eff(t_s) S          (banded stencil on rows)
//   k_dense_combine  k = Z + Z^ + sum_k L_k S L_k^ (32 x 32 tiles; Z^ read
//                    through LDS), fused with the RK4 stage update.
// rho stays exactly Hermitian: every stage derivative is formed as Z + Z^ + J
// with J symmetric by construction.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

struct DenseDev {
  int d_q, d_r, d_f, N;
  int frame;  // 1: frame rotating at w_d (mode frequencies already w - w_d)
  double w_q, alpha, w_r, w_f, g, G, kappa, gamma;
};

// Phase of a tap to a neighbour with dn more excitations in the drive frame:
// e^{-i w_d t dn}, from e1 = e^{i w_d t} and e2 = e^{2 i w_d t}.
__device__ __forceinline__ double2 tap_phase(int dn, double2 e1, double2 e2) {
  if (dn == 0) return make_double2(1.0, 0.0);
  const double2 e = (dn == 2 || dn == -2) ? e2 : e1;
  return dn < 0 ? e : make_double2(e.x, -e.y);
}

// mode indices of basis state n = (q d_r + r) d_f + f
__device__ __forceinline__ void dense_modes(const DenseDev& D, int n, int& q, int& r, int& f) {
  const int qr = n / D.d_f;
  f = n - qr * D.d_f;
  q = qr / D.d_r;
  r = qr - q * D.d_r;
}

constexpr int kDenseWG = 256;

// Z[a][b] = -i (H_eff S)[a][b] for one row a and 256 columns per workgroup.
// In the drive frame (D.frame) each coupling and drive tap carries
// tap_phase(dn) of the e1 = e^{i w_d t}, e2 = e^{2 i w_d t} of the stage.
__global__ __launch_bounds__(kDenseWG) void k_dense_apply(DenseDev D, double drv, double2 e1, double2 e2,
                                                          const double2* __restrict__ S, double2* __restrict__ Z) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * kDenseWG + threadIdx.x;
  if (b >= D.N) return;
  const int N = D.N, sf = 1, sr = D.d_f, sq = D.d_r * D.d_f;
  int q, r, f;
  dense_modes(D, a, q, r, f);
  const double hr = D.w_q * q + 0.5 * D.alpha * q * (q - 1) + D.w_r * r + D.w_f * f;
  const double hi = -0.5 * (D.kappa * f + D.gamma * q);
  const double2* col = S + b;
  double2 z = cmul(make_double2(hr, hi), col[(size_t)a * N]);
  // g (b + b^)(a + a^): q +- 1 with r +- 1
  for (int dq = -1; dq <= 1; dq += 2) {
    const int qq = q + dq;
    if (qq < 0 || qq >= D.d_q) continue;
    const double cq = sqrt((double)max(q, qq));
    for (int dr = -1; dr <= 1; dr += 2) {
      const int rr = r + dr;
      if (rr < 0 || rr >= D.d_r) continue;
      const double c = D.g * cq * sqrt((double)max(r, rr));
      const double2 nb = col[(size_t)(a + dq * sq + dr * sr) * N];
      z = D.frame ? cadd(z, cmul(cscale(c, tap_phase(dq + dr, e1, e2)), nb)) : cfma(c, nb, z);
    }
  }
  // G (a + a^)(f + f^) and the drive (f + f^)
  for (int df = -1; df <= 1; df += 2) {
    const int ff = f + df;
    if (ff < 0 || ff >= D.d_f) continue;
    const double cf = sqrt((double)max(f, ff));
    for (int dr = -1; dr <= 1; dr += 2) {
      const int rr = r + dr;
      if (rr < 0 || rr >= D.d_r) continue;
      const double c = D.G * cf * sqrt((double)max(r, rr));
      const double2 nb = col[(size_t)(a + dr * sr + df * sf) * N];
      z = D.frame ? cadd(z, cmul(cscale(c, tap_phase(dr + df, e1, e2)), nb)) : cfma(c, nb, z);
    }
    const double2 nb = col[(size_t)(a + df * sf) * N];
    z = D.frame ? cadd(z, cmul(cscale(drv * cf, tap_phase(df, e1, e2)), nb)) : cfma(drv * cf, nb, z);
  }
  Z[(size_t)a * N + b] = make_double2(z.y, -z.x);  // -i z
}

// sum_k (L_k S L_k^)[a][b] with L_1 = sqrt(kappa) f, L_2 = sqrt(gamma) b:
// c(a) c(b) S[a + e][b + e] for the shift e of the mode, where both exist.
__device__ __forceinline__ double2 dense_jumps(const DenseDev& D, const double2* S, int a, int b) {
  int qa, ra, fa, qb, rb, fb;
  dense_modes(D, a, qa, ra, fa);
  dense_modes(D, b, qb, rb, fb);
  double2 j = make_double2(0.0, 0.0);
  if (fa + 1 < D.d_f && fb + 1 < D.d_f) {
    const double c = D.kappa * sqrt((double)(fa + 1)) * sqrt((double)(fb + 1));
    j = cfma(c, S[(size_t)(a + 1) * D.N + (b + 1)], j);
  }
  const int sq = D.d_r * D.d_f;
  if (qa + 1 < D.d_q && qb + 1 < D.d_q) {
    const double c = D.gamma * sqrt((double)(qa + 1)) * sqrt((double)(qb + 1));
    j = cfma(c, S[(size_t)(a + sq) * D.N + (b + sq)], j);
  }
  return j;
}

// k = Z + Z^ + J and the RK4 stage update (stage s of 4):
//   s = 0: acc = k,        out = base + dt/2 k
//   s = 1: acc += 2 k,     out = base + dt/2 k
//   s = 2: acc += 2 k,     out = base + dt k
//   s = 3: base += dt/6 (acc + k), out = base
__global__ __launch_bounds__(kDenseWG) void k_dense_combine(DenseDev D, const double2* __restrict__ S,
                                                            const double2* __restrict__ Z, double2* __restrict__ base,
                                                            double2* __restrict__ acc, double2* __restrict__ out,
                                                            int s, double dt) {
  __shared__ double2 zt[32][33];
  const int N = D.N;
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // Z[b0 + i][a0 + j] -> zt[i][j]
  for (int i = ty; i < 32; i += 8) {
    const int rb = b0 + i, ca = a0 + tx;
    if (rb < N && ca < N) zt[i][tx] = Z[(size_t)rb * N + ca];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int a = a0 + i, b = b0 + tx;
    if (a >= N || b >= N) continue;
    const size_t o = (size_t)a * N + b;
    const double2 z = Z[o], zh = zt[tx][i];  // Z[a][b], Z[b][a]
    const double2 j = dense_jumps(D, S, a, b);
    const double2 k = make_double2(z.x + zh.x + j.x, z.y - zh.y + j.y);
    const double2 bo = base[o];
    double2 o_new;
    if (s == 0) {
      acc[o] = k;
      o_new = cfma(0.5 * dt, k, bo);
    } else if (s == 1) {
      acc[o] = cfma(2.0, k, acc[o]);
      o_new = cfma(0.5 * dt, k, bo);
    } else if (s == 2) {
      acc[o] = cfma(2.0, k, acc[o]);
      o_new = cfma(dt, k, bo);
    } else {
      o_new = cfma(dt / 6.0, cadd(acc[o], k), bo);
      base[o] = o_new;
    }
    if (s != 3) out[o] = o_new;
  }
}

// Observation record of a dense rho: [Re<a>, Im<a>, Re<f>, Im<f>, tr rho,
// tr rho^2, P_q(0..d_q-1)] (unnormalised tr(O rho)).  One workgroup, fixed
// order.
__global__ __launch_bounds__(kDenseWG) void k_dense_obs(DenseDev D, const double2* __restrict__ rho,
                                                        double* __restrict__ out) {
  __shared__ double red[kDenseWG];
  const int N = D.N, sr = D.d_f, sq = D.d_r * D.d_f;
  double v[6];
  for (int i = 0; i < 6; ++i) v[i] = 0.0;
  // <a> = sum_n sqrt(r+1) rho[n + e_r][n], <f> likewise, tr rho, tr rho^2
  for (int n = threadIdx.x; n < N; n += kDenseWG) {
    int q, r, f;
    dense_modes(D, n, q, r, f);
    if (r + 1 < D.d_r) {
      const double2 x = rho[(size_t)(n + sr) * N + n];
      v[0] += sqrt((double)(r + 1)) * x.x;
      v[1] += sqrt((double)(r + 1)) * x.y;
    }
    if (f + 1 < D.d_f) {
      const double2 x = rho[(size_t)(n + 1) * N + n];
      v[2] += sqrt((double)(f + 1)) * x.x;
      v[3] += sqrt((double)(f + 1)) * x.y;
    }
    v[4] += rho[(size_t)n * N + n].x;
  }
  for (size_t e = threadIdx.x; e < (size_t)N * N; e += kDenseWG) {
    const double2 x = rho[e];
    v[5] += x.x * x.x + x.y * x.y;  // tr rho^2 = sum |rho_ab|^2 (rho Hermitian)
  }
  for (int i = 0; i < 6 + D.d_q; ++i) {
    double x = 0.0;
    if (i < 6) {
      x = v[i];
    } else {
      const int k = i - 6;
      for (int n = k * sq + threadIdx.x; n < (k + 1) * sq; n += kDenseWG) x += rho[(size_t)n * N + n].x;
    }
    red[threadIdx.x] = x;
    __syncthreads();
    for (int off = kDenseWG / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

}  // namespace lrk
