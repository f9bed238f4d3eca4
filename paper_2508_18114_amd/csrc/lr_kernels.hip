// HIP kernels (gfx950) of the low-rank Lindblad RK4 integrator, FP64 path.
//
// One right-hand side evaluation of dB/dt = -i H_eff(t) B + 1/2 sum_k Y_k W_k,
// Y_k = L_k B, W_k = (G^-1 C_k)^, G = B^B, C_k = B^Y_k  (supplement S1.A,
// eq. "nosse" with the Moore-Penrose dissipator map) is split in two launches:
//
//   k_stage : one workgroup per tile of whole resonator layers.  Streams the
//             stage input through the banded operator (diagonal, transmon-
//             resonator and resonator-filter quadrature products, drive),
//             assembles the jump term with the W_k of this stage, applies the
//             RK4 stage update, and forms the Gram / cross-product partials of
//             the stage output over its own rows (the jumps stay in a layer).
//   k_solve : one workgroup per trajectory.  Reduces the partials in a fixed
//             tile order, factors G = R R^ (FP64 Cholesky), solves G X_k = C_k
//             and writes W_k = X_k^ for the next stage.
//
// Both launches are batched: a launch covers every tile (or trajectory) of a
// set of independent trajectories of possibly different shapes.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

// ----------------------------------------------------------------------------
// layout conversion between the ABI (column-major N x M, n = (q d_r + r) d_f + f)
// and the internal layer-major layout
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_to_internal(const TrajDev* __restrict__ trajs, int traj,
                                                     const double2* __restrict__ src,
                                                     double2* __restrict__ dst) {
  const TrajDev& T = trajs[traj];
  const int64_t total = (int64_t)T.N * T.M;
  for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < total; e += (int64_t)gridDim.x * kWG) {
    const int rho = (int)(e / T.M), j = (int)(e - (int64_t)rho * T.M);
    const int r = rho / T.L, rem = rho - r * T.L, q = rem / T.d_f, f = rem - q * T.d_f;
    const int n = (q * T.d_r + r) * T.d_f + f;
    dst[e] = src[(int64_t)j * T.N + n];
  }
}

__global__ __launch_bounds__(kWG) void k_to_abi(const TrajDev* __restrict__ trajs, int traj,
                                                const double2* __restrict__ src,
                                                double2* __restrict__ dst) {
  const TrajDev& T = trajs[traj];
  const int64_t total = (int64_t)T.N * T.M;
  for (int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x; e < total; e += (int64_t)gridDim.x * kWG) {
    const int j = (int)(e / T.N), n = (int)(e - (int64_t)j * T.N);
    const int q = n / (T.d_r * T.d_f), rem = n - q * T.d_r * T.d_f, r = rem / T.d_f, f = rem - r * T.d_f;
    const int rho = (r * T.d_q + q) * T.d_f + f;
    dst[e] = src[(int64_t)rho * T.M + j];
  }
}

// Reset the step counter and the error state of every trajectory of a batch.
__global__ void k_reset(const TrajDev* __restrict__ trajs, int ntraj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntraj) {
    *trajs[i].step = 0;
    *trajs[i].status = 0;
    *trajs[i].fail_step = -1;
  }
}

// Copy a by-value descriptor into device memory (graph- and stream-safe).
__global__ void k_set_traj(TrajDev* dst, TrajDev v) { *dst = v; }

__device__ __forceinline__ void report(const TrajDev& T, int code, int64_t step) {
  if (atomicCAS(T.status, 0, code) == 0) *T.fail_step = step;
}

// ----------------------------------------------------------------------------
// Gram / cross-product partials of the tile held in LDS (rows x M, row-major)
// ----------------------------------------------------------------------------
__device__ __forceinline__ void tile_gram_partials(const TrajDev& T, const double2* __restrict__ O,
                                                   int rows, int tile, double2* __restrict__ part) {
  const int M = T.M, MM = M * M, d_f = T.d_f, L = T.L;
  const double sk = sqrt(T.kappa), sg = sqrt(T.gamma);
  for (int o = threadIdx.x; o < MM; o += kWG) {
    const int i = o / M, j = o - i * M;
    double2 g = make_double2(0.0, 0.0), c1 = g, c2 = g;
    for (int rl = 0; rl < rows; ++rl) {
      const int rem = rl % L, q = rem / d_f, f = rem - q * d_f;
      const double2 oi = O[rl * M + i];
      g = cadd(g, cconjmul(oi, O[rl * M + j]));
      if (f + 1 < d_f) c1 = cadd(c1, cscale(sk * sqrt((double)(f + 1)), cconjmul(oi, O[(rl + 1) * M + j])));
      if (q + 1 < T.d_q) c2 = cadd(c2, cscale(sg * sqrt((double)(q + 1)), cconjmul(oi, O[(rl + d_f) * M + j])));
    }
    double2* P = part + (size_t)tile * 3 * MM;
    P[o] = g;
    P[MM + o] = c1;
    P[2 * MM + o] = c2;
  }
}

// ----------------------------------------------------------------------------
// stage kernel
//   mode MODE_STEP: RK4 stage s (0..3) of the current step of every trajectory
//   mode MODE_RHS : k = f(t0, Bb) written to acc (no partials)
//   mode MODE_GRAM: partials of Bb only
// tilemap[b] = (trajectory, tile index within it); r-range = tile*rt .. +rt
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_stage(const TrajDev* __restrict__ trajs,
                                               const int2* __restrict__ tilemap, const int* __restrict__ rt_of,
                                               int s, int mode) {
  extern __shared__ double2 lds[];
  const int2 tm = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tm.x];
  const int64_t step = *T.step;
  if (mode == MODE_STEP && step >= T.nsteps) return;

  const int M = T.M, MM = M * M, L = T.L, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const int rt = rt_of[tm.x];
  const int r0 = tm.y * rt, r1 = min(r0 + rt, d_r);
  const int row0 = r0 * L, rows = (r1 - r0) * L, E = rows * M;

  double2* ldsW = lds;            // 2 * M * M
  double2* ldsT = lds + 2 * MM;   // rows * M

  // stage buffers: s=0 Bb->S0, s=1 S0->S1, s=2 S1->S0, s=3 S0->Bb
  const double2* in;
  double2* out = nullptr;
  if (mode == MODE_GRAM || mode == MODE_RHS) {
    in = T.Bb;
  } else {
    in = (s == 0) ? T.Bb : (s == 2 ? T.S1 : T.S0);
    out = (s == 1) ? T.S1 : (s == 3 ? T.Bb : T.S0);
  }

  // stage tile (and W) into LDS
  for (int e = threadIdx.x; e < E; e += kWG) ldsT[e] = in[(size_t)row0 * M + e];
  if (mode != MODE_GRAM) {
    const double2* Wsrc = T.W + (size_t)(s & 1) * 2 * MM;
    for (int e = threadIdx.x; e < 2 * MM; e += kWG) ldsW[e] = Wsrc[e];
  }
  __syncthreads();

  if (mode == MODE_GRAM) {
    tile_gram_partials(T, ldsT, rows, tm.y, T.part);
    return;
  }

  const double cs = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);  // RK4 stage nodes 0, 1/2, 1/2, 1
  const double t = (mode == MODE_RHS) ? T.t0 : (T.t0 + (double)step * T.dt + cs * T.dt);
  const double drv = drive_at(T, t);
  // drive frame: a tap to a neighbour with dn more excitations carries e^{-i w_d t dn}
  const double2 e1 = frame_phase(T.w_d, t), e2 = frame_phase(2.0 * T.w_d, t);
  auto tap = [&](double2 z, double c, int dn, double2 nb) {
    if (!T.frame || dn == 0) return cfma(c, nb, z);
    const double2 e = (dn == 2 || dn == -2) ? e2 : e1;
    return cadd(z, cmul(cscale(c, dn < 0 ? e : make_double2(e.x, -e.y)), nb));
  };
  const double dt = T.dt;
  const double sk = sqrt(T.kappa), sg = sqrt(T.gamma);

#pragma unroll
  for (int k = 0; k < kMaxElemsPerThread; ++k) {
    const int e = threadIdx.x + k * kWG;
    if (e < E) {
    const int rl = e / M, j = e - rl * M;
    const int rho = row0 + rl;
    const int r = rho / L, rem = rho - r * L, q = rem / d_f, f = rem - q * d_f;
    const double2* col = in + j;
    const double2 b = ldsT[e];
    // diagonal of H_eff
    const double hr = T.w_q * q + 0.5 * T.alpha * q * (q - 1) + T.w_r * r + T.w_f * f;
    const double hi = -0.5 * (T.kappa * f + T.gamma * q);
    double2 z = cmul(make_double2(hr, hi), b);
    // g (b+b^)(a+a^): (q +- 1, r +- 1)
#pragma unroll
    for (int dq = -1; dq <= 1; dq += 2) {
      const int qq = q + dq;
      if (qq < 0 || qq >= d_q) continue;
      const double cq = sqrt((double)max(q, qq));
#pragma unroll
      for (int dr = -1; dr <= 1; dr += 2) {
        const int rr = r + dr;
        if (rr < 0 || rr >= d_r) continue;
        const double c = T.g * cq * sqrt((double)max(r, rr));
        z = tap(z, c, dq + dr, col[(size_t)(rho + dq * d_f + dr * L) * M]);
      }
    }
    // G (a+a^)(f+f^): (r +- 1, f +- 1); drive d(t) (f+f^): f +- 1
#pragma unroll
    for (int df = -1; df <= 1; df += 2) {
      const int ff = f + df;
      if (ff < 0 || ff >= d_f) continue;
      const double cf = sqrt((double)max(f, ff));
#pragma unroll
      for (int dr = -1; dr <= 1; dr += 2) {
        const int rr = r + dr;
        if (rr < 0 || rr >= d_r) continue;
        const double c = T.G * cf * sqrt((double)max(r, rr));
        z = tap(z, c, dr + df, col[(size_t)(rho + dr * L + df) * M]);
      }
      z = tap(z, drv * cf, df, ldsT[e + df * M]);
    }
    // jump assembly 1/2 sum_k (L_k B W_k)[rho, j]
    double2 a = make_double2(0.0, 0.0);
    if (f + 1 < d_f) {
      const double c = sk * sqrt((double)(f + 1));
      const double2* yr = ldsT + (rl + 1) * M;
      double2 acc1 = make_double2(0.0, 0.0);
      for (int i = 0; i < M; ++i) acc1 = cadd(acc1, cmul(yr[i], ldsW[i * M + j]));
      a = cfma(c, acc1, a);
    }
    if (q + 1 < d_q) {
      const double c = sg * sqrt((double)(q + 1));
      const double2* yr = ldsT + (rl + d_f) * M;
      double2 acc2 = make_double2(0.0, 0.0);
      for (int i = 0; i < M; ++i) acc2 = cadd(acc2, cmul(yr[i], ldsW[MM + i * M + j]));
      a = cfma(c, acc2, a);
    }
    // k = -i z + a/2
    const double2 kk = make_double2(z.y + 0.5 * a.x, -z.x + 0.5 * a.y);
    const size_t gi = (size_t)row0 * M + e;
    if (mode == MODE_RHS) {
      T.acc[gi] = kk;
    } else {
    double2 base = b;
    if (s != 0) base = T.Bb[gi];
    double2 o;
    if (s == 0) {
      T.acc[gi] = kk;
      o = cfma(0.5 * dt, kk, base);
    } else if (s == 1) {
      T.acc[gi] = cfma(2.0, kk, T.acc[gi]);
      o = cfma(0.5 * dt, kk, base);
    } else if (s == 2) {
      T.acc[gi] = cfma(2.0, kk, T.acc[gi]);
      o = cfma(dt, kk, base);
    } else {
      o = cfma(dt / 6.0, cadd(T.acc[gi], kk), base);
    }
    out[gi] = o;
    }
    }
  }
  if (mode == MODE_RHS) return;

  __syncthreads();  // every thread is done reading the stage input tile
  // the stage output of this tile replaces it in LDS (each thread re-reads its
  // own global writes, which are ordered before these loads)
#pragma unroll
  for (int k = 0; k < kMaxElemsPerThread; ++k) {
    const int e = threadIdx.x + k * kWG;
    if (e < E) ldsT[e] = out[(size_t)row0 * M + e];
  }
  __syncthreads();
  tile_gram_partials(T, ldsT, rows, tm.y, T.part);
}

// ----------------------------------------------------------------------------
// solve kernel: one workgroup per trajectory
//   reduce partials -> G, C_1, C_2 ; ||G||_F^2 ; Cholesky G = R R^ ;
//   X_k = G^-1 C_k ; W_k = X_k^  into W[wpar]
//   advance != 0: increment the step counter afterwards (end of an RK step)
//   mode MODE_GRAM: reduce and record ||G||_F^2 only (observables of any B)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_solve(const TrajDev* __restrict__ trajs, int wpar, int advance,
                                               int mode) {
  __shared__ double2 A[kMaxM * kMaxM];
  __shared__ double2 Cc[kMaxM * 2 * kMaxM];
  __shared__ double red[kWG];
  __shared__ int bad;
  const TrajDev& T = trajs[blockIdx.x];
  const int64_t step = *T.step;
  if (mode == MODE_STEP && step >= T.nsteps) return;
  const int M = T.M, MM = M * M, M2 = 2 * M, nt = T.ntiles;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();

  // fixed-order reduction of the tile partials
  double fro = 0.0;
  int nonfinite = 0;
  for (int o = tid; o < 3 * MM; o += kWG) {
    const int m = o / MM, ij = o - m * MM;
    double2 acc = make_double2(0.0, 0.0);
    for (int t = 0; t < nt; ++t) acc = cadd(acc, T.part[(size_t)t * 3 * MM + o]);
    if (!isfinite(acc.x) || !isfinite(acc.y)) nonfinite = 1;
    const int i = ij / M, j = ij - i * M;
    if (m == 0) {
      A[ij] = acc;
      fro += acc.x * acc.x + acc.y * acc.y;
    } else {
      Cc[i * M2 + (m - 1) * M + j] = acc;
    }
  }
  red[tid] = fro;
  if (nonfinite) atomicOr(&bad, 1);
  __syncthreads();
  for (int w = kWG / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const bool advance_here = advance && mode == MODE_STEP;
  if (tid == 0) *T.fro2 = red[0];
  if (bad) {
    if (tid == 0) {
      report(T, -5 /* LR_ERR_NONFINITE */, step);
      if (advance_here) *T.step = step + 1;
    }
    return;
  }
  if (mode == MODE_GRAM) return;

  // Cholesky G = R R^ (R lower, in A) with the right-hand sides carried
  // along, i.e. the forward substitution R Y = [C_1 C_2] fused in.
  for (int k = 0; k < M; ++k) {
    const double piv = A[k * M + k].x;
    if (!(piv > 0.0)) {
      if (tid == 0) {
        report(T, -4 /* LR_ERR_GRAM_NOT_PD */, step);
        if (advance_here) *T.step = step + 1;
      }
      return;  // uniform: every thread read the same pivot after a barrier
    }
    const double d = sqrt(piv), inv = 1.0 / d;
    const int nr = M - k - 1;
    for (int o = tid; o < nr + M2; o += kWG) {
      if (o < nr) {
        const int i = k + 1 + o;
        A[i * M + k] = cscale(inv, A[i * M + k]);
      } else {
        const int c = o - nr;
        Cc[k * M2 + c] = cscale(inv, Cc[k * M2 + c]);
      }
    }
    __syncthreads();
    if (tid == 0) A[k * M + k] = make_double2(d, 0.0);
    for (int o = tid; o < nr * nr + nr * M2; o += kWG) {
      if (o < nr * nr) {
        const int i = k + 1 + o / nr, j = k + 1 + o % nr;
        if (j <= i) {
          const double2 u = cmulc(A[i * M + k], A[j * M + k]);  // L_ik conj(L_jk)
          A[i * M + j] = make_double2(A[i * M + j].x - u.x, A[i * M + j].y - u.y);
        }
      } else {
        const int oo = o - nr * nr;
        const int i = k + 1 + oo / M2, c = oo % M2;
        const double2 u = cmul(A[i * M + k], Cc[k * M2 + c]);
        Cc[i * M2 + c] = make_double2(Cc[i * M2 + c].x - u.x, Cc[i * M2 + c].y - u.y);
      }
    }
    __syncthreads();
  }
  // back substitution R^ X = Y (X overwrites Y)
  for (int k = M - 1; k >= 0; --k) {
    const double inv = 1.0 / A[k * M + k].x;
    for (int c = tid; c < M2; c += kWG) Cc[k * M2 + c] = cscale(inv, Cc[k * M2 + c]);
    __syncthreads();
    for (int o = tid; o < k * M2; o += kWG) {
      const int i = o / M2, c = o - i * M2;
      const double2 u = cconjmul(A[k * M + i], Cc[k * M2 + c]);  // conj(L_ki) X_kc
      Cc[i * M2 + c] = make_double2(Cc[i * M2 + c].x - u.x, Cc[i * M2 + c].y - u.y);
    }
    __syncthreads();
  }
  // W_k[i][j] = conj(X_k[j][i])
  double2* Wd = T.W + (size_t)wpar * 2 * MM;
  for (int o = tid; o < 2 * MM; o += kWG) {
    const int kk = o / MM, ij = o - kk * MM, i = ij / M, j = ij - i * M;
    const double2 x = Cc[j * M2 + kk * M + i];
    Wd[o] = make_double2(x.x, -x.y);
  }
  if (advance_here && tid == 0) *T.step = step + 1;
}

// ----------------------------------------------------------------------------
// observables: one workgroup per trajectory, fixed-order block reductions.
//   rec: [Re<a>, Im<a>, Re<f>, Im<f>, tr rho, tr rho^2, P_q(0..d_q-1)]
//   dst == null: record into T.obs at index step / obs_stride when
//   step % obs_stride == 0 (during an integration); else write to dst.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = kWG / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kWG) void k_obs(const TrajDev* __restrict__ trajs, double* dst) {
  __shared__ double red[kWG];
  const TrajDev& T = trajs[blockIdx.x];
  const int64_t step = *T.step;
  double* rec = dst;
  if (rec == nullptr) {
    if (T.obs == nullptr || T.obs_stride <= 0 || step > T.nsteps || step % T.obs_stride != 0) return;
    rec = T.obs + (size_t)(step / T.obs_stride) * (6 + T.d_q);
  }
  const int M = T.M, L = T.L, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const double2* B = T.Bb;
  const int per_q = d_r * d_f * M;  // elements with a given transmon level
  double ar = 0.0, ai = 0.0, fr = 0.0, fi = 0.0, tr = 0.0;
  for (int q = 0; q < d_q; ++q) {
    double pq = 0.0;
    for (int e = threadIdx.x; e < per_q; e += kWG) {
      const int r = e / (d_f * M), rem = e - r * d_f * M, f = rem / M, j = rem - f * M;
      const int rho = (r * d_q + q) * d_f + f;
      const double2 v = B[(size_t)rho * M + j];
      const double p = v.x * v.x + v.y * v.y;
      pq += p;
      if (r + 1 < d_r) {
        const double2 u = cconjmul(v, B[(size_t)(rho + L) * M + j]);
        const double c = sqrt((double)(r + 1));
        ar = fma(c, u.x, ar);
        ai = fma(c, u.y, ai);
      }
      if (f + 1 < d_f) {
        const double2 u = cconjmul(v, B[(size_t)(rho + 1) * M + j]);
        const double c = sqrt((double)(f + 1));
        fr = fma(c, u.x, fr);
        fi = fma(c, u.y, fi);
      }
    }
    tr += pq;
    const double s = block_sum(pq, red);
    if (threadIdx.x == 0) rec[6 + q] = s;
  }
  const double s_ar = block_sum(ar, red), s_ai = block_sum(ai, red);
  double s_fr = block_sum(fr, red), s_fi = block_sum(fi, red);
  const double s_tr = block_sum(tr, red);
  if (T.mkind == 2) {
    // normal-mode basis: the filter field f = s21 c_u^ + s22 c_l^ + s23 c_l + s24 c_u (supplement S2.D)
    // from the mode fields <c_l> (resonator slot) and <c_u> (filter slot); in the drive frame the
    // creation terms carry e^{2 i w_d t} (the record is e^{i w_d t} times the lab-frame field, as for
    // the other kinds)
    double2 e2 = make_double2(1.0, 0.0);
    if (T.frame) {
      const double2 e1 = frame_phase(T.w_d, T.t0 + (double)(T.step_base + step) * T.dt);
      e2 = cmul(e1, e1);
    }
    const double2 cl = make_double2(s_ar, s_ai), cu = make_double2(s_fr, s_fi);
    const double2 cr = make_double2(T.nm[0] * cu.x + T.nm[1] * cl.x, -(T.nm[0] * cu.y + T.nm[1] * cl.y));
    const double2 an = make_double2(T.nm[2] * cl.x + T.nm[3] * cu.x, T.nm[2] * cl.y + T.nm[3] * cu.y);
    const double2 fv = cadd(an, cmul(e2, cr));
    s_fr = fv.x;
    s_fi = fv.y;
  }
  if (threadIdx.x == 0) {
    rec[0] = s_ar;
    rec[1] = s_ai;
    rec[2] = s_fr;
    rec[3] = s_fi;
    rec[4] = s_tr;
    rec[5] = *T.fro2;
  }
}

}  // namespace lrk
