// Spectrum of the low-rank density matrix: the eigenvalues p_1 >= ... >= p_M
// of G = B^ B, which are the nonzero eigenvalues of rho = B B^ (the weights
// of eq. "lowrank_diagonal").  Supplement S1.B uses p_M / p_1 as the control
// quantity of the approximation, and the purity tr rho^2 = sum_j p_j^2.
//
// One workgroup per state:
//   1. G = B^ B in FP64 from the caller's column-major N x M layout: blocks
//      of kSpecRows rows are staged in LDS, and each thread accumulates its
//      entries (i, j) over the rows in order.
//   2. The Hermitian G is embedded as the real symmetric 2M x 2M matrix
//      S = [[Re G, -Im G], [Im G, Re G]], whose spectrum is that of G with
//      every eigenvalue twice, and S is diagonalised by cyclic Jacobi
//      rotations (the symmetric Schur decomposition of a 2 x 2 block per
//      pivot pair).  A sweep visits every pair once in the round-robin order:
//      each of its 2M - 1 rounds rotates M disjoint pairs together (all row
//      rotations, then all column rotations).  Sweeps repeat until the
//      off-diagonal part is below 1e-32 of ||S||_F^2, or has stopped falling
//      (less than halved by a sweep: the rounding floor), at most kSpecSweeps.
//   3. The 2M diagonal values are sorted in descending order and averaged in
//      pairs.
// Every step has a fixed order, so the result depends on the input only.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

constexpr int kSpecWG = 256;
constexpr int kSpecRows = 32;    // rows of B staged per block
constexpr int kSpecSweeps = 30;
constexpr int kSpecMaxM = 32;

__global__ __launch_bounds__(kSpecWG) void k_spectrum(const double2* __restrict__ B, int N, int M,
                                                       double* __restrict__ out) {
  __shared__ double2 blk[kSpecRows * kSpecMaxM];
  __shared__ double S[4 * kSpecMaxM * kSpecMaxM];
  __shared__ double rc[kSpecMaxM], rs[kSpecMaxM];
  __shared__ int rp[kSpecMaxM], rq[kSpecMaxM];
  __shared__ double red[kSpecWG];
  __shared__ int s_done;
  const int tid = threadIdx.x, MM = M * M, K = 2 * M;

  // 1. G = B^ B; thread t owns entries t, t + kSpecWG, ... (at most 4)
  double2 g[4];
  for (int u = 0; u < 4; ++u) g[u] = make_double2(0.0, 0.0);
  for (int r0 = 0; r0 < N; r0 += kSpecRows) {
    const int nr = min(kSpecRows, N - r0);
    __syncthreads();
    for (int idx = tid; idx < nr * M; idx += kSpecWG) {
      const int j = idx / nr, r = idx - j * nr;  // column-major: consecutive threads read consecutive rows
      blk[r * M + j] = B[(size_t)j * N + r0 + r];
    }
    __syncthreads();
    for (int u = 0; u < 4; ++u) {
      const int o = tid + u * kSpecWG;
      if (o < MM) {
        const int i = o / M, j = o - i * M;
        for (int r = 0; r < nr; ++r) g[u] = cjmac(g[u], blk[r * M + i], blk[r * M + j]);
      }
    }
  }
  // 2. S = [[Re G, -Im G], [Im G, Re G]]
  for (int u = 0; u < 4; ++u) {
    const int o = tid + u * kSpecWG;
    if (o < MM) {
      const int i = o / M, j = o - i * M;
      S[i * K + j] = g[u].x;
      S[(i + M) * K + j + M] = g[u].x;
      S[i * K + j + M] = -g[u].y;
      S[(i + M) * K + j] = g[u].y;
    }
  }
  __syncthreads();
  double fro = 0.0;  // ||S||_F^2, fixed-order block sum
  {
    double v = 0.0;
    for (int e = tid; e < K * K; e += kSpecWG) v += S[e] * S[e];
    red[tid] = v;
    __syncthreads();
    for (int off = kSpecWG / 2; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    fro = red[0];
    __syncthreads();
  }
  const int npair = M;  // K / 2 disjoint pairs per round
  double prev = fro;
  for (int sweep = 0; sweep < kSpecSweeps; ++sweep) {
    for (int round = 0; round < K - 1; ++round) {
      // round-robin: position 0 stays, positions 1 .. K-1 rotate by `round`
      if (tid < npair) {
        const int x = tid, y = K - 1 - tid;
        const int a = x == 0 ? 0 : (x - 1 + round) % (K - 1) + 1;
        const int b = (y - 1 + round) % (K - 1) + 1;
        const int p = min(a, b), q = max(a, b);
        const double apq = S[p * K + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (S[q * K + q] - S[p * K + p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
      }
      __syncthreads();
      // rows: row_p <- c row_p - s row_q, row_q <- s row_p + c row_q
      for (int e = tid; e < npair * K; e += kSpecWG) {
        const int k = e / K, col = e - k * K;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], s = rs[k];
        const double xp = S[p * K + col], xq = S[q * K + col];
        S[p * K + col] = c * xp - s * xq;
        S[q * K + col] = s * xp + c * xq;
      }
      __syncthreads();
      // columns: col_p <- c col_p - s col_q, col_q <- s col_p + c col_q
      for (int e = tid; e < npair * K; e += kSpecWG) {
        const int k = e / K, row = e - k * K;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], s = rs[k];
        const double xp = S[row * K + p], xq = S[row * K + q];
        S[row * K + p] = c * xp - s * xq;
        S[row * K + q] = s * xp + c * xq;
      }
      __syncthreads();
    }
    double v = 0.0;
    for (int e = tid; e < K * K; e += kSpecWG) {
      const int i = e / K, j = e - i * K;
      if (i != j) v += S[e] * S[e];
    }
    red[tid] = v;
    __syncthreads();
    for (int off = kSpecWG / 2; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    const double off = red[0];
    // (a non-finite G ends here too)
    if (tid == 0) s_done = !(off > 1e-32 * fro) || (sweep > 0 && off > 0.5 * prev);
    prev = off;
    __syncthreads();
    if (s_done) break;
  }
  // 3. descending order of the diagonal (in red), then pair averages
  if (tid < K) red[tid] = S[tid * K + tid];
  __syncthreads();
  if (tid == 0) {
    double* d = red;
    for (int i = 1; i < K; ++i) {
      const double x = d[i];
      int k = i - 1;
      while (k >= 0 && d[k] < x) {
        d[k + 1] = d[k];
        --k;
      }
      d[k + 1] = x;
    }
    for (int k = 0; k < M; ++k) out[k] = 0.5 * (d[2 * k] + d[2 * k + 1]);
  }
}

}  // namespace lrk
