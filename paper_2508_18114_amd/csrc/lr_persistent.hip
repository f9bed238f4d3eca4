// Persistent on-chip RK4 integrator (gfx950).
//
// A trajectory is split into P workgroups, each owning `rt` whole resonator
// layers (the jump operators never leave a layer).  The state of a workgroup's
// rows -- the base B_n and the RK4 accumulator in registers, the current stage
// input in LDS -- stays on chip for a whole chunk of steps.  Per RK4 stage:
//
//   1. solve G X_k = C_k for the reduced G = S^S, C_k = S^ L_k S of the stage
//      input (FP64 elimination of the augmented [G | C_1 C_2] in registers,
//      one pivot per barrier); W_k = X_k^
//   2. k_s = -i H_eff(t_s) S + 1/2 sum_k (L_k S) W_k for the own rows (banded
//      stencil with one halo layer up and down, jump assembly), RK4 stage
//      update in registers
//   3. Gram / cross partials of the new stage input over the own rows;
//      publish them and the two boundary layers
//   4. group barrier A; halo layers in; reduce a 1/P slice of the partials
//      (fixed order); group barrier B
//
// Cross-workgroup data moves through agent-coherent (sc1) loads and stores;
// group barriers are per-workgroup release flags polled with acquire
// semantics (no shared counter).  Every wait is bounded: an expired wait
// raises a per-trajectory abort flag that ends the whole group.  The launch is
// cooperative, so all workgroups of a group are co-resident.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

constexpr int kPW = 512;  // threads per workgroup
// The kernel is instantiated for ROWS = 2 and 3 rows of one column per
// thread (ceil(rows / (kPW / M)) <= ROWS); 2 keeps every value in registers.
constexpr int kMaxRowsPerThread = 3;
constexpr size_t kPersistLdsMax = 159 * 1024;  // dynamic LDS (160 KB less the static part)

// Dynamic LDS bytes of k_persist for rt layers of L rows at rank M and P
// workgroups: stage input with halos, W, slice-reduction buffer, pivot
// row/column (double buffered), per-row jump coefficients.
__host__ __device__ inline size_t persist_lds_bytes(int rt, int L, int M, int P) {
  return (size_t)((rt + 2) * L * M + 2 * M * M + 3 * M * M + P + 2 * 4 * M) * 16 + (size_t)2 * rt * L * 8;
}

// agent-coherent 16-byte store / load (two 64-bit atomic accesses)
__device__ __forceinline__ void st_ag(g_double2* p, double2 v) {
  g_double* d = reinterpret_cast<g_double*>(p);
  __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_ag(const g_double2* p) {
  const g_double* d = reinterpret_cast<const g_double*>(p);
  return make_double2(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// plain 16-byte global load / store through a global-address-space pointer
__device__ __forceinline__ double2 ld_g(const g_double2* p) {
  const g_double* d = reinterpret_cast<const g_double*>(p);
  return make_double2(d[0], d[1]);
}
__device__ __forceinline__ void st_g(g_double2* p, double2 v) {
  g_double* d = reinterpret_cast<g_double*>(p);
  d[0] = v.x;
  d[1] = v.y;
}

__device__ __forceinline__ void flag_arrive(g_u32* flag, uint32_t value) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until flags[w * kFlagStride] >= target for all w < P.  Returns false
// if the wait expired or the group was aborted.
__device__ __forceinline__ bool flag_wait(const TrajDev& T, const g_u32* flags, uint32_t target, int* s_ok) {
  g_u32* abort_flag = (g_u32*)T.abort_flag;
  if (threadIdx.x < 64) {
    bool ok = true;
    for (int w = threadIdx.x; w < T.P && ok; w += 64) {
      uint32_t n = 0;
      while (__hip_atomic_load(flags + (size_t)w * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             target) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++n > kSpinLimit) {
          __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const bool all_ok = __all(ok);
    if (threadIdx.x == 0) *s_ok = all_ok ? 1 : 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return *s_ok != 0;
}

// Publish the two boundary layers of the tile (rows [0, L) and [R-L, R)).
__device__ __forceinline__ void publish_boundary(const double2* tile, g_double2* dst, int row0, int R, int L, int M) {
  const int LM = L * M;
  for (int idx = threadIdx.x; idx < 2 * LM; idx += kPW) {
    const int off = idx < LM ? idx : (R - L) * M + (idx - LM);
    st_ag(dst + (size_t)row0 * M + off, tile[off]);
  }
}

// Gram / cross partials of the tile (rows x M in LDS) -> dst[3 M^2]:
//   G[i][j]   = sum_rho conj(O[rho][i]) O[rho][j]
//   C_1[i][j] = sum_rho conj(O[rho][i]) sqrt(kappa (f+1)) O[rho+1][j]      (f+1 < d_f)
//   C_2[i][j] = sum_rho conj(O[rho][i]) sqrt(gamma (q+1)) O[rho+d_f][j]    (q+1 < d_q)
// c1row / c2row hold those coefficients per row and 0 where the jump leaves
// the mode (the row read there is a finite neighbour in the tile or halo).
// With PAIR, rows are taken in pairs with separate accumulators (fixed
// order either way).
template <bool PAIR>
__device__ __forceinline__ void persist_partials(const TrajDev& T, const double2* tile, int R, const double* c1row,
                                                 const double* c2row, g_double2* dst) {
  const int M = T.M, MM = M * M, d_f = T.d_f;
  for (int o = threadIdx.x; o < MM; o += kPW) {
    const int i = o / M, jj = o - i * M;
    double2 g0 = make_double2(0.0, 0.0), a10 = g0, a20 = g0, g1 = g0, a11 = g0, a21 = g0;
    int rl = 0;
    if (PAIR)
    for (; rl + 2 <= R; rl += 2) {
      const double2 oi0 = tile[rl * M + i], oi1 = tile[(rl + 1) * M + i];
      const double2 oj0 = tile[rl * M + jj], oj1 = tile[(rl + 1) * M + jj];
      const double2 f0 = tile[(rl + 1) * M + jj], f1 = tile[(rl + 2) * M + jj];
      const double2 q0 = tile[(rl + d_f) * M + jj], q1 = tile[(rl + 1 + d_f) * M + jj];
      const double c10 = c1row[rl], c11 = c1row[rl + 1], c20 = c2row[rl], c21 = c2row[rl + 1];
      g0 = cadd(g0, cconjmul(oi0, oj0));
      g1 = cadd(g1, cconjmul(oi1, oj1));
      a10 = cfma(c10, cconjmul(oi0, f0), a10);
      a11 = cfma(c11, cconjmul(oi1, f1), a11);
      a20 = cfma(c20, cconjmul(oi0, q0), a20);
      a21 = cfma(c21, cconjmul(oi1, q1), a21);
    }
    for (; rl < R; ++rl) {
      const double2 oi0 = tile[rl * M + i];
      g0 = cadd(g0, cconjmul(oi0, tile[rl * M + jj]));
      a10 = cfma(c1row[rl], cconjmul(oi0, tile[(rl + 1) * M + jj]), a10);
      a20 = cfma(c2row[rl], cconjmul(oi0, tile[(rl + d_f) * M + jj]), a20);
    }
    st_ag(dst + o, cadd(g0, g1));
    st_ag(dst + MM + o, cadd(a10, a11));
    st_ag(dst + 2 * MM + o, cadd(a20, a21));
  }
}

// Reciprocal of a positive FP64 pivot: hardware estimate refined by two
// Newton steps (r <- r + r (1 - p r)), accurate to about an ulp.
__device__ __forceinline__ double pivot_rcp(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  r = fma(r, fma(-p, r, 1.0), r);
  return r;
}

// W_k = X_k^ with X_k = G^-1 C_k (G Hermitian positive definite), in two
// parallel phases:
//   1. in-place Gauss-Jordan inversion of G without pivoting: M pivot steps,
//      each a rank-1 update of every entry from the pivot row and column (one
//      barrier per pivot).  Its pivots are those of the Cholesky factorisation
//      G = L D L^ (D_k > 0 iff G is positive definite); a non-positive pivot
//      is reported like a failed Cholesky.
//   2. W_k[i][j] = sum_l conj(C_k[l][i]) (G^-1)[l][j]  (= (G^-1 C_k)^ since
//      G^-1 is Hermitian), every entry independent.
// G entries live in registers (thread t owns flat entries t, t + kPW);
// C_k and G^-1 go through LDS.  solve_load issues the loads of the reduced
// G, C_k so that their latency overlaps other work; solve_run finishes.
constexpr int kGE = 2;  // ceil(M^2 / kPW) for M <= 32
constexpr int kCE = 4;  // ceil(2 M^2 / kPW)

struct SolveRegs {
  double2 g[kGE];
  double2 c[kCE];
};

__device__ __forceinline__ void solve_load(const g_double2* red, int M, SolveRegs& S) {
  const int MM = M * M;
#pragma unroll
  for (int u = 0; u < kGE; ++u) S.g[u] = ld_ag(red + min((int)threadIdx.x + u * kPW, MM - 1));
#pragma unroll
  for (int u = 0; u < kCE; ++u) S.c[u] = ld_ag(red + MM + min((int)threadIdx.x + u * kPW, 2 * MM - 1));
}

// Cs (2 M^2) and Gi (M^2) are LDS scratch; prow, pcol hold 2 x M each.
// Writes W_k to Wl.  Returns -1, the first non-positive pivot, or -2 for a
// non-finite input.
__device__ __forceinline__ int solve_run(SolveRegs& S, double2* prow, double2* pcol, double2* Cs, double2* Gi,
                                         double2* Wl, int M, int* nonfinite_flag) {
  const int MM = M * M;
  const int tid = threadIdx.x;
  int bad_local = 0;
#pragma unroll
  for (int u = 0; u < kGE; ++u)
    if (tid + u * kPW < MM && (!isfinite(S.g[u].x) || !isfinite(S.g[u].y))) bad_local = 1;
#pragma unroll
  for (int u = 0; u < kCE; ++u) {
    const int o = tid + u * kPW;
    if (o < 2 * MM) {
      if (!isfinite(S.c[u].x) || !isfinite(S.c[u].y)) bad_local = 1;
      Cs[o] = S.c[u];
    }
  }
  if (tid == 0) *nonfinite_flag = 0;
  __syncthreads();
  if (bad_local) *nonfinite_flag = 1;
  __syncthreads();
  if (*nonfinite_flag) return -2;

  int gi[kGE], gj[kGE];
#pragma unroll
  for (int u = 0; u < kGE; ++u) {
    const int o = min(tid + u * kPW, MM - 1);
    gi[u] = o / M;
    gj[u] = o - gi[u] * M;
  }
  const int nu = (MM + kPW - 1) / kPW;
  for (int k = 0; k < M; ++k) {
    double2* pr = prow + (k & 1) * M;
    double2* pc = pcol + (k & 1) * M;
#pragma unroll
    for (int u = 0; u < kGE; ++u) {
      if (u < nu && tid + u * kPW < MM) {
        if (gi[u] == k) pr[gj[u]] = S.g[u];
        if (gj[u] == k) pc[gi[u]] = S.g[u];
      }
    }
    __syncthreads();
    const double piv = pr[k].x;
    if (!(piv > 0.0)) return k;  // uniform: every thread read the same pivot
    const double inv = pivot_rcp(piv);
#pragma unroll
    for (int u = 0; u < kGE; ++u) {
      if (u < nu) {
        const double2 a = pc[gi[u]], bkj = pr[gj[u]];
        const bool ri = gi[u] == k, cj = gj[u] == k;
        double2 v;
        if (ri && cj) v = make_double2(inv, 0.0);
        else if (ri) v = cscale(inv, S.g[u]);
        else if (cj) v = cscale(-inv, S.g[u]);
        else {
          const double2 t = cscale(inv, cmul(a, bkj));
          v = make_double2(S.g[u].x - t.x, S.g[u].y - t.y);
        }
        S.g[u] = v;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kGE; ++u)
    if (tid + u * kPW < MM) Gi[tid + u * kPW] = S.g[u];
  __syncthreads();
  // W_k[i][j] = sum_l conj(C_k[l][i]) Gi[l][j]
  for (int o = tid; o < 2 * MM; o += kPW) {
    const int kk = o / MM, ij = o - kk * MM, i = ij / M, j = ij - i * M;
    const double2* C = Cs + kk * MM;
    double2 s0 = make_double2(0.0, 0.0), s1 = s0;
    int l = 0;
    for (; l + 2 <= M; l += 2) {
      s0 = cadd(s0, cconjmul(C[l * M + i], Gi[l * M + j]));
      s1 = cadd(s1, cconjmul(C[(l + 1) * M + i], Gi[(l + 1) * M + j]));
    }
    if (l < M) s0 = cadd(s0, cconjmul(C[l * M + i], Gi[l * M + j]));
    Wl[o] = cadd(s0, s1);
  }
  __syncthreads();
  return -1;
}

// Sum of |G_ij|^2 over the reduced Gram (block reduction, fixed order).
__device__ __forceinline__ double gram_fro2(const g_double2* red, int MM, double* s_part) {
  double v = 0.0;
  for (int o = threadIdx.x; o < MM; o += kPW) {
    const double2 g = ld_ag(red + o);
    v += g.x * g.x + g.y * g.y;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kPW / 64; ++w) tot += s_part[w];
  __syncthreads();
  return tot;
}

template <int ROWS>
__global__ __launch_bounds__(kPW) void k_persist(const TrajDev* __restrict__ trajs,
                                                 const int2* __restrict__ tilemap, int prologue, int64_t step0,
                                                 int64_t nchunk) {
  extern __shared__ double2 lds[];
  __shared__ int s_ok;
  __shared__ int s_nonfinite;
  __shared__ double s_part[kPW / 64];

  const int2 tm = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tm.x];
  const int w = tm.y, P = T.P;
  const int M = T.M, MM = M * M, L = T.L, d_q = T.d_q, d_r = T.d_r, d_f = T.d_f;
  const int rt = T.rt, r0 = w * rt, r1 = min(r0 + rt, d_r);
  const int R = (r1 - r0) * L, row0 = r0 * L, LM = L * M;
  const int npe = T.npe;
  const int tid = threadIdx.x;
  g_double2* Bb = (g_double2*)T.Bb;
  g_double2* SPg = (g_double2*)T.SP;
  g_double2* PARTg = (g_double2*)T.PART;
  g_double2* REDg = (g_double2*)T.RED;

  // dynamic LDS layout
  double2* SL = lds;                              // (rt + 2) L M: [halo | tile | halo]
  double2* tile = SL + LM;
  double2* Wl = SL + (size_t)(rt + 2) * LM;       // 2 M^2
  double2* RB = Wl + 2 * MM;                      // 3 M^2 + P   (slice reduction)
  double2* prow = RB + 3 * MM + P;                // 2 x 3M
  double2* pcol = prow + 6 * M;                   // 2 x M
  double* c1row = reinterpret_cast<double*>(pcol + 2 * M);
  double* c2row = c1row + rt * L;

  // halo layers start at zero: the jump partials read one neighbour row past
  // the tile edge with a zero coefficient
  for (int idx = tid; idx < 2 * LM; idx += kPW) SL[idx < LM ? idx : (size_t)(R + L) * M + (idx - LM)] = make_double2(0.0, 0.0);
  for (int rl = tid; rl < R; rl += kPW) {
    const int rem = rl % L, q = rem / d_f, f = rem - q * d_f;
    c1row[rl] = f + 1 < d_f ? sqrt(T.kappa * (double)(f + 1)) : 0.0;
    c2row[rl] = q + 1 < d_q ? sqrt(T.gamma * (double)(q + 1)) : 0.0;
  }

  // element mapping: column j, rows rg, rg + NG, ...
  const int NG = kPW / M;
  const int j = tid % M, rg = tid / M;
  const bool active = rg < NG;

  double2 base[ROWS], acc[ROWS], o_new[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int rl = rg + k * NG;
    base[k] = make_double2(0.0, 0.0);
    acc[k] = base[k];
    o_new[k] = base[k];
    if (active && rl < R) {
      base[k] = ld_g(Bb + (size_t)(row0 + rl) * M + j);
      tile[rl * M + j] = base[k];
    }
  }
  g_u32* flagA = (g_u32*)T.flagA;
  g_u32* flagB = (g_u32*)T.flagB;
  g_u32* myA = flagA + (size_t)w * kFlagStride;
  g_u32* myB = flagB + (size_t)w * kFlagStride;
  const int64_t NMn = (int64_t)T.N * M;
  const int cs = (npe + P - 1) / P;
  const int e0 = w * cs, e1 = min(npe, e0 + cs), ne = max(0, e1 - e0);

  // slice reduction of the partials of parity `par`: all loads in flight at
  // once into LDS, then a fixed-order sum over the workgroups per entry
  auto reduce_slice = [&](int par) {
    const g_double2* src = PARTg + (size_t)par * P * npe;
    const int nit = ne * P;
    for (int base_it = 0; base_it < nit; base_it += 4 * kPW) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int it = min(base_it + tid + u * kPW, nit - 1);
        const int pp = it / ne, e = it - pp * ne;
        v[u] = ld_ag(src + (size_t)pp * npe + e0 + e);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int it = base_it + tid + u * kPW;
        if (it < nit) RB[it] = v[u];
      }
    }
    __syncthreads();
    g_double2* dst = REDg + (size_t)par * npe + e0;
    for (int e = tid; e < ne; e += kPW) {
      double2 s = make_double2(0.0, 0.0);
      for (int pp = 0; pp < P; ++pp) s = cadd(s, RB[pp * ne + e]);
      st_ag(dst + e, s);
    }
  };
  auto load_halo = [&](int par) {
    const g_double2* src = SPg + (size_t)par * NMn;
    const size_t lo_base = r0 > 0 ? (size_t)(row0 - L) * M : 0;
    const size_t hi_base = r1 < d_r ? (size_t)(row0 + R) * M : 0;
    for (int base_idx = 0; base_idx < 2 * LM; base_idx += 4 * kPW) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = min(base_idx + tid + u * kPW, 2 * LM - 1);
        const bool lo = idx < LM;
        const int off = lo ? idx : idx - LM;
        v[u] = ld_ag(src + (lo ? lo_base : hi_base) + off);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = base_idx + tid + u * kPW;
        if (idx < 2 * LM) {
          const bool lo = idx < LM;
          const int off = lo ? idx : idx - LM;
          const bool have = lo ? r0 > 0 : r1 < d_r;
          const double2 val = have ? v[u] : make_double2(0.0, 0.0);
          if (lo) SL[off] = val;
          else SL[(size_t)(R + L) * M + off] = val;
        }
      }
    }
  };

  if (prologue) {
    const int64_t g = 4 * step0;
    const int p = (int)(g & 1);
    __syncthreads();
    persist_partials<ROWS == 2>(T, tile, R, c1row, c2row, PARTg + ((size_t)p * P + w) * npe);
    publish_boundary(tile, SPg + (size_t)p * NMn, row0, R, L, M);
    flag_arrive(myA, (uint32_t)(g + 1));
    bool ok = flag_wait(T, flagA, (uint32_t)(g + 1), &s_ok);
    if (ok) {
      reduce_slice(p);
      flag_arrive(myB, (uint32_t)(g + 1));
      ok = flag_wait(T, flagB, (uint32_t)(g + 1), &s_ok);
    }
    if (!ok) {
      if (tid == 0) report(T, -8 /* LR_ERR_TIMEOUT */, step0);
      return;
    }
    if (w == 0) {
      const double f2 = gram_fro2(REDg + (size_t)p * npe, MM, s_part);
      if (tid == 0) {
        *T.fro2 = f2;
        *T.step = step0;
      }
    }
    return;
  }

  // chunk: the reduction of stage 4*step0 and the published boundary layers
  // of its input are in global memory
  load_halo((int)((4 * step0) & 1));
  const double dt = T.dt;
  const int64_t nrun = max((int64_t)0, min(nchunk, T.nsteps - step0));  // trajectories of a batch end apart
  bool ok = true;
  bool failed = false;
  int64_t n = 0;
  for (; n < nrun && ok && !failed; ++n) {
    const int64_t step = step0 + n;
    for (int s = 0; s < 4; ++s) {
      const int64_t g = 4 * step + s;
      const int p = (int)(g & 1);
      const double cs_ = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);
      const double t = T.t0 + (double)step * dt + cs_ * dt;
      const double drv = drive_at(T, t);
      __syncthreads();  // stage input tile and halo in LDS

      // (1) loads of the reduced G, C_k in flight while Z = H_eff(t) S is formed
      SolveRegs SR;
      solve_load(REDg + (size_t)p * npe, M, SR);
      double2 z[ROWS];
#pragma unroll
      for (int k = 0; k < ROWS; ++k) {
        const int rl = rg + k * NG;
        z[k] = make_double2(0.0, 0.0);
        if (active && rl < R) {
          const int rho = row0 + rl;
          const int r = rho / L, rem = rho - r * L, q = rem / d_f, f = rem - q * d_f;
          const double2* col = tile + j;  // row offsets relative to the tile (halo at -L, +R)
          const double2 b = col[rl * M];
          const double hr = T.w_q * q + 0.5 * T.alpha * q * (q - 1) + T.w_r * r + T.w_f * f;
          const double hi = -0.5 * (T.kappa * f + T.gamma * q);
          double2 zz = cmul(make_double2(hr, hi), b);
          for (int dq = -1; dq <= 1; dq += 2) {
            const int qq = q + dq;
            if (qq < 0 || qq >= d_q) continue;
            const double cq = sqrt((double)max(q, qq));
            for (int dr = -1; dr <= 1; dr += 2) {
              const int rr = r + dr;
              if (rr < 0 || rr >= d_r) continue;
              zz = cfma(T.g * cq * sqrt((double)max(r, rr)), col[(rl + dq * d_f + dr * L) * M], zz);
            }
          }
          for (int df = -1; df <= 1; df += 2) {
            const int ff = f + df;
            if (ff < 0 || ff >= d_f) continue;
            const double cf = sqrt((double)max(f, ff));
            for (int dr = -1; dr <= 1; dr += 2) {
              const int rr = r + dr;
              if (rr < 0 || rr >= d_r) continue;
              zz = cfma(T.G * cf * sqrt((double)max(r, rr)), col[(rl + dr * L + df) * M], zz);
            }
            zz = cfma(drv * cf, col[(rl + df) * M], zz);
          }
          z[k] = zz;
        }
      }
      // (2) W_k of this stage input
      {
        const int bad = solve_run(SR, prow, pcol, RB, RB + 2 * MM, Wl, M, &s_nonfinite);
        if (bad != -1) {
          if (tid == 0) report(T, bad == -2 ? -5 /* LR_ERR_NONFINITE */ : -4 /* LR_ERR_GRAM_NOT_PD */, step);
          failed = true;
          break;
        }
      }

      // (3) k = -i Z + 1/2 sum_k (L_k S) W_k ; RK4 stage update
#pragma unroll
      for (int k = 0; k < ROWS; ++k) {
        const int rl = rg + k * NG;
        if (active && rl < R) {
          const double2 zz = z[k];
          // jump assembly: c1 (S W_1)[rho+1, j] + c2 (S W_2)[rho+d_f, j]; the
          // coefficient is 0 where the jump leaves the mode
          const double2* y1 = tile + (rl + 1) * M;
          const double2* y2 = tile + (rl + d_f) * M;
          const double2* W1 = Wl + j;
          const double2* W2 = Wl + MM + j;
          double2 s1a = make_double2(0.0, 0.0), s1b = s1a, s2a = s1a, s2b = s1a;
          int i = 0;
          // two accumulator pairs where registers allow (three rows per thread
          // would spill)
          if (ROWS == 2)
          for (; i + 2 <= M; i += 2) {
            s1a = cadd(s1a, cmul(y1[i], W1[i * M]));
            s1b = cadd(s1b, cmul(y1[i + 1], W1[(i + 1) * M]));
            s2a = cadd(s2a, cmul(y2[i], W2[i * M]));
            s2b = cadd(s2b, cmul(y2[i + 1], W2[(i + 1) * M]));
          }
          for (; i < M; ++i) {
            s1a = cadd(s1a, cmul(y1[i], W1[i * M]));
            s2a = cadd(s2a, cmul(y2[i], W2[i * M]));
          }
          const double2 a = cfma(c2row[rl], cadd(s2a, s2b), cscale(c1row[rl], cadd(s1a, s1b)));
          const double2 kk = make_double2(zz.y + 0.5 * a.x, -zz.x + 0.5 * a.y);
          double2 o;
          if (s == 0) {
            acc[k] = kk;
            o = cfma(0.5 * dt, kk, base[k]);
          } else if (s == 1) {
            acc[k] = cfma(2.0, kk, acc[k]);
            o = cfma(0.5 * dt, kk, base[k]);
          } else if (s == 2) {
            acc[k] = cfma(2.0, kk, acc[k]);
            o = cfma(dt, kk, base[k]);
          } else {
            base[k] = cfma(dt / 6.0, cadd(acc[k], kk), base[k]);
            o = base[k];
          }
          o_new[k] = o;
        }
      }
      __syncthreads();  // every thread is done reading the stage input
#pragma unroll
      for (int k = 0; k < ROWS; ++k) {
        const int rl = rg + k * NG;
        if (active && rl < R) tile[rl * M + j] = o_new[k];
      }
      __syncthreads();

      // (4) partials and boundary layers of the next stage input
      const int pn = p ^ 1;
      persist_partials<ROWS == 2>(T, tile, R, c1row, c2row, PARTg + ((size_t)pn * P + w) * npe);
      publish_boundary(tile, SPg + (size_t)pn * NMn, row0, R, L, M);

      // (5) group barriers around the slice reduction
      flag_arrive(myA, (uint32_t)(g + 2));
      ok = flag_wait(T, flagA, (uint32_t)(g + 2), &s_ok);
      if (!ok) break;
      load_halo(pn);
      reduce_slice(pn);
      flag_arrive(myB, (uint32_t)(g + 2));
      ok = flag_wait(T, flagB, (uint32_t)(g + 2), &s_ok);
      if (!ok) break;
    }
  }
  if (!ok && tid == 0) report(T, -8 /* LR_ERR_TIMEOUT */, step0 + n);

  // state out
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int rl = rg + k * NG;
    if (active && rl < R) st_g(Bb + (size_t)(row0 + rl) * M + j, base[k]);
  }
  if (w == 0 && ok && !failed && nrun > 0) {
    const double f2 = gram_fro2(REDg, MM, s_part);  // parity of stage 4 (step0 + nrun) is 0
    if (tid == 0) {
      *T.fro2 = f2;
      *T.step = step0 + nrun;
    }
  } else if (w == 0 && tid == 0) {
    *T.step = step0 + n;
  }
}

// Zero the barrier flags and the abort flag of every trajectory of a batch.
__global__ void k_reset_persist(const TrajDev* __restrict__ trajs, int ntraj) {
  if ((int)blockIdx.x >= ntraj) return;
  const TrajDev& T = trajs[blockIdx.x];
  for (int i = threadIdx.x; i < T.P * kFlagStride; i += blockDim.x) {
    T.flagA[i] = 0u;
    T.flagB[i] = 0u;
  }
  if (threadIdx.x == 0) *T.abort_flag = 0u;
}

}  // namespace lrk
