// Packed schedule of a batch: one workgroup integrates one whole trajectory.
//
// The persistent kernel spreads a trajectory over one workgroup per resonator
// layer and pays, every stage, two device-wide flag barriers and a redundant
// M x M solve in each workgroup: the shortest time per step, but a CU holds
// one of those workgroups, so a batch runs about 256 / d_r trajectories at a
// time.  Here a workgroup owns a trajectory for the whole launch and streams
// its layers in order; nothing crosses workgroups, so every CU holds as many
// trajectories as its LDS and registers allow and a batch fills the chip.
//
// Per RK4 stage (the right-hand side of eq. "nosse", supplement S1.A):
//   for each resonator layer r (L = d_q d_f rows x M columns):
//     1. layers r - 1, r, r + 1 of the stage input Y are in LDS (each loaded
//        while the Gram terms of an earlier layer were formed); each element
//        takes the H_eff stencil, the jump assembly 1/2 sum_k (L_k Y)[rho, :]
//        W_k[:, j] against the W_k in LDS, and the RK4 combination with B_n
//        and the accumulator (loaded during the assembly); the stage output
//        goes to global memory and to a fourth LDS tile;
//     2. every thread adds the layer's contribution to its own entries of
//        [G | C_1 | C_2] = O^ [O | L_1 O | L_2 O] of the stage output O (the
//        jumps stay in a layer), rows in order;
//   then the M x 3M matrix [G | C_1 | C_2] goes to LDS and Gauss-Jordan
//   elimination without pivoting turns it into [I | G^-1 C_1 | G^-1 C_2]
//   (the pivots are those of G = L D L^; the pivot is the real part of the
//   diagonal entry, as G is Hermitian), which gives W_k = (G^-1 C_k)^ of the
//   next stage.
// Every sum has a fixed order, so a trajectory's result does not depend on
// the batch it runs in.  The rounding differs from the persistent kernel's
// (another summation order and another elimination), within the FP64
// tolerances of the oracle comparison.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

constexpr int kTW = 256;            // threads of a packed workgroup
constexpr int kTMaxLM = 1536;       // rows x M of one layer
constexpr size_t kPackedLdsMax = 159 * 1024;  // dynamic LDS of one workgroup (of 160 KiB per CU)
constexpr int kTRowBlock = 2;       // layer rows per thread per assembly pass
constexpr int kTPrefetch = 5;       // elements per thread of the next layer held in registers
constexpr int kTDriveWin = 32;      // steps per drive table refill

// LDS (in complex elements) of a packed workgroup: four layer tiles (three
// layers of the stage input, one of the output), or the M x 3M elimination
// matrix; W_1, W_2; the drive table (kTDriveWin steps x 4 stages x 5 doubles)
// and the pivot row of the elimination (3M); per-row tables (jump
// coefficients and the diagonal of H_eff without its resonator term, 5 L
// doubles) and sqrt(0 .. dmax), dmax = max(d_q, d_r, d_f).
__host__ __device__ inline size_t packed_lds_elems(int L, int M, int dmax) {
  const size_t tiles = 4 * (size_t)L * M, aug = 3 * (size_t)M * M;
  // (+16: the Gram-term row blocks may read up to 15 elements past the output tile)
  return (tiles > aug ? tiles : aug) + 2 * (size_t)M * M + 10 * kTDriveWin + 3 * (size_t)M +
         (5 * (size_t)L + dmax + 2) / 2 + 16;
}
// Entries of [G | C_1 | C_2] per thread: thread t owns column t mod 3M and
// the block of KPe consecutive rows from (t / 3M) KPe, KPe = ceil(M / NG),
// NG = 256 / (3M) row groups.  Kernel variants exist for a few block sizes
// KP >= KPe (the entries past KPe are computed and dropped).
__host__ __device__ inline int packed_kpe(int M) {
  const int ng = kTW / (3 * M);
  return (M + ng - 1) / ng;
}
inline int packed_kp(int M) {
  const int need = packed_kpe(M);
  return need <= 2 ? 2 : need <= 3 ? 3 : need <= 5 ? 5 : need <= 8 ? 8 : need <= 12 ? 12 : 16;
}

// Element (rl, j) of layer r: H_eff stencil and drive on the stage input
// (own layer in LDS, neighbour layers from global memory); returns z = H_eff Y.
// Gram terms of one layer tile O for K consecutive rows of [G | C_1 | C_2]
// from pi0, column pcc of [O | L_1 O | L_2 O]: acc[k] += sum_rl conj(O[rl][pi0
// + k]) cr[rl] O[rl + shift][pcc] (cr = 0 where the jump leaves the
// truncation; its source row is clamped into the tile).
template <int K, int KP>
__device__ __forceinline__ void gram_rows(double2 (&acc)[KP], const double2* Ot, const double* cr, int L, int M,
                                          int shift, int pcc, int pi0) {
  for (int rl = 0; rl < L; ++rl) {
    const double2 x = cscale(cr[rl], Ot[min(rl + shift, L - 1) * M + pcc]);
    const double2* o = Ot + rl * M + pi0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = cjmac(acc[k], o[k], x);
  }
}

// Mapping of a packed workgroup's threads onto [G | C_1 | C_2] (M x 3M): thread
// t owns column pc = t mod 3M of [O | L_1 O | L_2 O] (pkind 0, 1, 2 = G, filter,
// transmon; pcc its column within) and rows pi0 .. pi0 + KPe - 1.
struct PackedMap {
  int M, C3, L, d_f, KPe, pc, pi0, pkind, pcc;
  bool pact;
};

// Gram terms of the layer tile Ot, added to the thread's entries (the block
// size KPe is uniform: one branch picks the unrolled loop).
template <int KP>
__device__ __forceinline__ void packed_terms(double2 (&acc)[KP], const PackedMap& P, const double2* Ot,
                                             const double* coef) {
  if (!P.pact) return;
  const int L = P.L, M = P.M, KPe = P.KPe, pcc = P.pcc, pi0 = P.pi0;
  const int shift = P.pkind == 0 ? 0 : (P.pkind == 1 ? 1 : P.d_f);
  const double* cr = coef + P.pkind * L;
  if (KPe <= 2 || KP == 2) {
    gram_rows<2>(acc, Ot, cr, L, M, shift, pcc, pi0);
  } else if (KPe <= 3 || KP == 3) {
    if constexpr (KP >= 3) gram_rows<3>(acc, Ot, cr, L, M, shift, pcc, pi0);
  } else if (KPe <= 5 || KP == 5) {
    if constexpr (KP >= 5) gram_rows<5>(acc, Ot, cr, L, M, shift, pcc, pi0);
  } else if (KPe <= 8 || KP == 8) {
    if constexpr (KP >= 8) gram_rows<8>(acc, Ot, cr, L, M, shift, pcc, pi0);
  } else if (KPe <= 12 || KP == 12) {
    if constexpr (KP >= 12) gram_rows<12>(acc, Ot, cr, L, M, shift, pcc, pi0);
  } else {
    if constexpr (KP >= 16) gram_rows<16>(acc, Ot, cr, L, M, shift, pcc, pi0);
  }
}

// [G | C_1 | C_2] (the threads' entries) -> W_1, W_2 in Wl, through the M x 3M
// elimination in Aug; returns 0, or -4 (pivot <= 0) / -5 (non-finite).
template <int KP>
__device__ __forceinline__ int packed_solve(double2 (&acc)[KP], const PackedMap& P, double2* Aug, double2* Wl,
                                            double2* s_prow, double* s_red, int* s_flag, bool want_fro2,
                                            double* fro2) {
  const int tid = threadIdx.x, M = P.M, MM = M * M, C3 = P.C3, KPe = P.KPe, pi0 = P.pi0, pc = P.pc;
  const bool pact = P.pact;
  const int pkind = P.pkind;
  __syncthreads();  // the tiles are free
  int bad = 0;
  double f2 = 0.0;
  if (pact) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = pi0 + k;
      if (k < KPe && i < M) {
        Aug[i * C3 + pc] = acc[k];
        if (!isfinite(acc[k].x) || !isfinite(acc[k].y)) bad = 1;
        if (pkind == 0) f2 += acc[k].x * acc[k].x + acc[k].y * acc[k].y;
      }
    }
  }
  if (tid == 0) *s_flag = 0;
  __syncthreads();
  if (bad) *s_flag = 1;
  if (want_fro2) {
    for (int off = 32; off > 0; off >>= 1) f2 += __shfl_xor(f2, off);
    if ((tid & 63) == 0) s_red[tid >> 6] = f2;
  }
  __syncthreads();
  if (want_fro2) {
    double tot = 0.0;
    for (int w = 0; w < kTW / 64; ++w) tot += s_red[w];
    *fro2 = tot;
  }
  if (*s_flag) return -5;
  // pivot p: the scaled pivot row goes to s_prow, then every entry right of
  // the pivot column takes x - Aug[i][p] prow[c] (the pivot row: prow[c]);
  // the pivot column is only read
  const int tot = M * C3;
  for (int p = 0; p < M; ++p) {
    const double piv = Aug[p * C3 + p].x;
    if (!(piv > 0.0)) return -4;
    const double rp = pivot_rcp(piv);
    for (int c = p + 1 + tid; c < C3; c += kTW) s_prow[c] = cscale(rp, Aug[p * C3 + c]);
    __syncthreads();
    for (int e = tid; e < tot; e += kTW) {
      const int i = e / C3, c = e - i * C3;
      if (c > p) {
        const double2 pr = s_prow[c];
        if (i == p) {
          Aug[e] = pr;
        } else {
          const double2 l = Aug[i * C3 + p];
          Aug[e] = cadd(Aug[e], cmul(make_double2(-l.x, -l.y), pr));
        }
      }
    }
    __syncthreads();
  }
  // W_k[i][j] = conj(X_k[j][i]), X_k = columns M (k + 1) .. of the eliminated matrix
  for (int e = tid; e < 2 * MM; e += kTW) {
    const int k = e / MM, o = e - k * MM, i = o / M, j = o - i * M;
    const double2 x = Aug[j * C3 + M * (k + 1) + i];
    Wl[e] = make_double2(x.x, -x.y);
  }
  __syncthreads();
  return 0;
}

// Element (rl, j) of layer r: z = H_eff Y (stencil and drive) from the layers
// r - 1, r, r + 1 of the stage input in LDS (Yp, Yc, Yn).  sq[k] = sqrt(k);
// hd[rl] = diagonal of H_eff at row rl without w_r r.
template <bool ROT>
__device__ __forceinline__ double2 packed_stencil(const TrajDev& T, const double2* Yp, const double2* Yc,
                                                  const double2* Yn, const double* sq, const double2* hd, int r,
                                                  int rl, int q, int f, int j, double drv, double2 e1, double2 e2) {
  const int M = T.M, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const double2 b = Yc[rl * M + j];
  auto tap = [&](double2 z, double c, int dn, double2 nb) {
    if (!ROT || dn == 0) return cfma(c, nb, z);
    const double2 e = (dn == 2 || dn == -2) ? e2 : e1;
    return cadd(z, cmul(cscale(c, dn < 0 ? e : make_double2(e.x, -e.y)), nb));
  };
  const double2 h = hd[rl];
  double2 z = cmul(make_double2(h.x + T.w_r * r, h.y), b);
  const double sr_lo = sq[r], sr_hi = sq[min(r + 1, d_r)];
#pragma unroll
  for (int dq = -1; dq <= 1; dq += 2) {
    const int qq = q + dq;
    if (qq < 0 || qq >= d_q) continue;
    const double cq = T.g * sq[max(q, qq)];
    if (r > 0) z = tap(z, cq * sr_lo, dq - 1, Yp[(rl + dq * d_f) * M + j]);
    if (r + 1 < d_r) z = tap(z, cq * sr_hi, dq + 1, Yn[(rl + dq * d_f) * M + j]);
  }
#pragma unroll
  for (int df = -1; df <= 1; df += 2) {
    const int ff = f + df;
    if (ff < 0 || ff >= d_f) continue;
    const double cf = sq[max(f, ff)];
    if (r > 0) z = tap(z, T.G * cf * sr_lo, df - 1, Yp[(rl + df) * M + j]);
    if (r + 1 < d_r) z = tap(z, T.G * cf * sr_hi, df + 1, Yn[(rl + df) * M + j]);
    z = tap(z, drv * cf, df, Yc[(rl + df) * M + j]);
  }
  return z;
}

// Element (rl, j) of layer r for the transmon-eigenbasis model:
// z = H Y with H = diag(E_q + w_r r + w_f f) - i/2 (jumps) + i g n_t (a^ - a)
// - J (a^ - a)(f^ - f) + d(t) i (f^ - f), J held in T.G.  (a^ Y)[r] = sqrt(r)
// Y[r-1], (a Y)[r] = sqrt(r+1) Y[r+1]; n_t couples the transmon levels densely
// (row q of nt, from LDS).  ROT: the frame rotating at w_d (levels and mode
// frequencies already reduced by w_d in hd and T); a tap from a neighbour with
// dn more excitations (level index + n_r + n_f) carries e^{-i w_d t dn}, read
// as the conjugate of ph[dn + ph0] = e^{i w_d t dn}.
template <bool ROT>
__device__ __forceinline__ double2 packed_stencil_tm(const TrajDev& T, const double2* Yp, const double2* Yc,
                                                     const double2* Yn, const double* sq, const double2* hd,
                                                     const double* nt, const double2* ph, int ph0, int r, int rl,
                                                     int q, int f, int j, double drv) {
  const int M = T.M, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const double2 h = hd[rl];
  double2 z = cmul(make_double2(h.x + T.w_r * r, h.y), Yc[rl * M + j]);
  const double sr_lo = sq[r], sr_hi = sq[min(r + 1, d_r)];
  // c nb, phased by e^{-i w_d t dn} in the rotating frame
  auto tap = [&](double2 acc, double c, int dn, double2 nb) {
    if (!ROT || dn == 0) return cfma(c, nb, acc);
    const double2 e = ph[dn + ph0];
    return cadd(acc, cmul(make_double2(c * e.x, -c * e.y), nb));
  };
  // i g n_t (a^ - a)
  double2 s = make_double2(0.0, 0.0);
  for (int p = 0; p < d_q; ++p) {
    const double c = nt[q * d_q + p];
    if (c == 0.0) continue;
    const int row = p * d_f + f;
    if (r > 0) s = tap(s, c * sr_lo, p - q - 1, Yp[row * M + j]);
    if (r + 1 < d_r) s = tap(s, -c * sr_hi, p - q + 1, Yn[row * M + j]);
  }
  z = make_double2(z.x - T.g * s.y, z.y + T.g * s.x);
  // -J (a^ - a)(f^ - f), and d(t) i (f^ - f)
  double2 u = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
#pragma unroll
  for (int df = -1; df <= 1; df += 2) {
    const int ff = f + df;
    if (ff < 0 || ff >= d_f) continue;
    const double cf = (df < 0 ? 1.0 : -1.0) * sq[max(f, ff)];
    if (r > 0) u = tap(u, cf * sr_lo, df - 1, Yp[(rl + df) * M + j]);
    if (r + 1 < d_r) u = tap(u, -cf * sr_hi, df + 1, Yn[(rl + df) * M + j]);
    v = tap(v, cf, df, Yc[(rl + df) * M + j]);
  }
  z = cfma(-T.G, u, z);
  return make_double2(z.x - drv * v.y, z.y + drv * v.x);
}

// The kernel body: prologue (Gram terms and W of the initial state, no step)
// or a chunk of nchunk RK4 steps from step0.  KP = entries of [G|C_1|C_2] per
// thread (packed_kp).
template <int KP, bool ROT, int MK = 0>
__device__ __forceinline__ void packed_body(const TrajDev& T, int prologue, int64_t step0, int64_t nchunk) {
  extern __shared__ double2 lds[];
  __shared__ double s_red[kTW / 64];
  __shared__ double s_nt[kMaxDq * kMaxDq];
  __shared__ double2 s_ph[2 * kMaxDq + 3];  // e^{i w_d t m}, m = -(d_q + 1) .. d_q + 1, of the stage (kind 1, rotating frame)
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int M = T.M, MM = M * M, L = T.L, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const int LM = L * M, C3 = 3 * M;
  const double dt = T.dt;
  const double sk = sqrt(T.kappa), sg = sqrt(T.gamma);
  double2* Yp = lds;                                  // layers r - 1, r, r + 1 of the stage input
  double2* Yc = lds + LM;
  double2* Yn = lds + 2 * LM;
  double2* Ot = lds + 3 * LM;                         // layer r of the stage output
  double2* Aug = lds;                                 // M x 3M elimination (after the layer loop)
  double2* Wl = lds + (4 * LM > 3 * MM ? 4 * LM : 3 * MM);  // W_1, W_2 (M x M each, row i, column j)
  double (*s_dtab)[5] = reinterpret_cast<double (*)[5]>(Wl + 2 * MM);  // [4 kTDriveWin][5] drive table
  double2* s_prow = Wl + 2 * MM + 10 * kTDriveWin;          // [3M] pivot row
  double2* hd = s_prow + 3 * M;                             // [L] diagonal of H_eff without w_r r
  double* coef = reinterpret_cast<double*>(hd + L);         // [3][L]: 1, filter jump, transmon jump
  double* sq = coef + 3 * L;                                // sqrt(0 .. dmax)
  g_double2* gBb = (g_double2*)T.Bb;
  g_double2* gacc = (g_double2*)T.acc;
  g_double2* gW = (g_double2*)T.W;

  if (tid == 0) s_flag = *T.status;
  if constexpr (MK == 1)
    for (int i = tid; i < d_q * d_q; i += kTW) s_nt[i] = T.ntq[i];
  for (int rl = tid; rl < L; rl += kTW) {
    const int q = rl / d_f, f = rl - q * d_f;
    const double eq = MK == 1 ? T.Et[q] - (ROT ? T.w_d * q : 0.0) : T.w_q * q + 0.5 * T.alpha * q * (q - 1);
    hd[rl] = make_double2(eq + T.w_f * f, -0.5 * (T.kappa * f + T.gamma * q));
    coef[rl] = 1.0;
    coef[L + rl] = (f + 1 < d_f) ? sk * sqrt((double)(f + 1)) : 0.0;
    coef[2 * L + rl] = (q + 1 < d_q) ? sg * sqrt((double)(q + 1)) : 0.0;
  }
  for (int k = tid; k <= max(max(d_q, d_r), d_f); k += kTW) sq[k] = sqrt((double)k);
  __syncthreads();
  if (s_flag != 0) return;
  const int64_t nrun = prologue ? 0 : (step0 < T.nsteps ? min(nchunk, T.nsteps - step0) : 0);
  if (!prologue && nrun <= 0) return;

  // element mapping: column j, rows g, g + NGe, ...
  const int NGe = kTW / M;
  const int ej = tid % M, eg = tid / M;
  const bool eact = eg < NGe;
  // Gram-term mapping: column c of [O | L_1 O | L_2 O], rows i = pi0 + k
  const int NGp = kTW / C3, KPe = packed_kpe(M);
  const int pc = tid % C3, pg = tid / C3, pi0 = pg * KPe;
  const bool pact = pg < NGp && pi0 < M;
  const int pkind = pc / M, pcc = pc - pkind * M;  // 0: G, 1: C_1 (filter), 2: C_2 (transmon)

  if (!prologue)
    for (int e = tid; e < 2 * MM; e += kTW) Wl[e] = ld_g(gW + e);

  auto stage_time = [&](int64_t step, int s) {
    const double c = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);
    return T.t0 + (double)(T.step_base + step) * dt + c * dt;
  };
  auto fill_drive = [&](int64_t step) {
    __syncthreads();
    if (tid < 4 * kTDriveWin) {
      const double t = stage_time(step + tid / 4, tid % 4);
      s_dtab[tid][0] = drive_at(T, t);
      const double2 p1 = frame_phase(T.w_d, t), p2 = frame_phase(2.0 * T.w_d, t);
      s_dtab[tid][1] = p1.x;
      s_dtab[tid][2] = p1.y;
      s_dtab[tid][3] = p2.x;
      s_dtab[tid][4] = p2.y;
    }
    __syncthreads();
  };

  const PackedMap PM{M, C3, L, d_f, KPe, pc, pi0, pkind, pcc, pact};
  auto add_terms = [&](double2 (&acc)[KP]) { packed_terms<KP>(acc, PM, Ot, coef); };
  auto solve = [&](double2 (&acc)[KP], bool want_fro2, double* fro2) -> int {
    return packed_solve<KP>(acc, PM, Aug, Wl, s_prow, s_red, &s_flag, want_fro2, fro2);
  };

  double2 acc[KP];

  if (prologue) {
#pragma unroll
    for (int k = 0; k < KP; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int r = 0; r < d_r; ++r) {
      __syncthreads();
      for (int e = tid; e < LM; e += kTW) Ot[e] = ld_g(gBb + (size_t)r * LM + e);
      __syncthreads();
      add_terms(acc);
    }
    double f2 = 0.0;
    const int rc = solve(acc, true, &f2);
    if (rc) {
      if (tid == 0) report(T, rc, step0);
      return;
    }
    for (int e = tid; e < 2 * MM; e += kTW) st_g(gW + e, Wl[e]);
    if (tid == 0) {
      *T.fro2 = f2;
      *T.step = step0;
    }
    return;
  }

  for (int64_t n = 0; n < nrun; ++n) {
    const int64_t step = step0 + n;
    if (n % kTDriveWin == 0) fill_drive(step);
    for (int s = 0; s < 4; ++s) {
      const g_double2* in = (const g_double2*)((s == 0) ? T.Bb : (s == 2 ? T.S1 : T.S0));
      g_double2* out = (g_double2*)((s == 1) ? T.S1 : (s == 3 ? T.Bb : T.S0));
      const int ds = (int)(n % kTDriveWin) * 4 + s;
      const double drv = s_dtab[ds][0];
      const double2 e1 = make_double2(s_dtab[ds][1], s_dtab[ds][2]), e2 = make_double2(s_dtab[ds][3], s_dtab[ds][4]);
#pragma unroll
      for (int k = 0; k < KP; ++k) acc[k] = make_double2(0.0, 0.0);
      if constexpr (MK == 1 && ROT)
        if (tid < 2 * d_q + 3) s_ph[tid] = frame_phase((tid - d_q - 1) * T.w_d, stage_time(step, s));
      __syncthreads();  // Wl of this stage written; tiles free
      Yp = lds;
      Yc = lds + LM;
      Yn = lds + 2 * LM;
      for (int e = tid; e < LM; e += kTW) Yc[e] = ld_g(in + e);
      if (d_r > 1)
        for (int e = tid; e < LM; e += kTW) Yn[e] = ld_g(in + LM + e);
      __syncthreads();
      for (int r = 0; r < d_r; ++r) {
        // 1. stage output of layer r, in blocks of kTRowBlock rows per thread
        if (eact) {
          for (int rb = eg; rb < L; rb += kTRowBlock * NGe) {
            // B_n and the RK4 accumulator of the block are in flight during the jump assembly
            double2 pb[kTRowBlock], pa[kTRowBlock];
            if (s > 0) {
#pragma unroll
              for (int k = 0; k < kTRowBlock; ++k) {
                const int rl = min(rb + k * NGe, L - 1);
                const size_t gi = ((size_t)r * L + rl) * M + ej;
                pb[k] = ld_g(gBb + gi);
                pa[k] = ld_g(gacc + gi);
              }
            }
            double2 a1[kTRowBlock], a2[kTRowBlock];
            int s1[kTRowBlock], s2[kTRowBlock];  // source rows of the jumps, clamped into the tile
#pragma unroll
            for (int k = 0; k < kTRowBlock; ++k) {
              a1[k] = a2[k] = make_double2(0.0, 0.0);
              const int rl = min(rb + k * NGe, L - 1);
              s1[k] = min(rl + 1, L - 1) * M;
              s2[k] = min(rl + d_f, L - 1) * M;
            }
            for (int i = 0; i < M; ++i) {
              const double2 w1 = Wl[i * M + ej], w2 = Wl[MM + i * M + ej];
#pragma unroll
              for (int k = 0; k < kTRowBlock; ++k) {
                a1[k] = cmac(a1[k], Yc[s1[k] + i], w1);
                a2[k] = cmac(a2[k], Yc[s2[k] + i], w2);
              }
            }
#pragma unroll
            for (int k = 0; k < kTRowBlock; ++k) {
              const int rl = rb + k * NGe;
              if (rl < L) {
                const int q = rl / d_f, f = rl - q * d_f;
                const double2 a = cfma(coef[L + rl], a1[k], cscale(coef[2 * L + rl], a2[k]));
                double2 z;
                if constexpr (MK == 1)
                  z = packed_stencil_tm<ROT>(T, Yp, Yc, Yn, sq, hd, s_nt, s_ph, d_q + 1, r, rl, q, f, ej, drv);
                else
                  z = packed_stencil<ROT>(T, Yp, Yc, Yn, sq, hd, r, rl, q, f, ej, drv, e1, e2);
                const double2 kk = make_double2(z.y + 0.5 * a.x, -z.x + 0.5 * a.y);
                const size_t gi = ((size_t)r * L + rl) * M + ej;
                double2 o;
                if (s == 0) {
                  st_g(gacc + gi, kk);
                  o = cfma(0.5 * dt, kk, Yc[rl * M + ej]);
                } else if (s == 1) {
                  st_g(gacc + gi, cfma(2.0, kk, pa[k]));
                  o = cfma(0.5 * dt, kk, pb[k]);
                } else if (s == 2) {
                  st_g(gacc + gi, cfma(2.0, kk, pa[k]));
                  o = cfma(dt, kk, pb[k]);
                } else {
                  o = cfma(dt / 6.0, cadd(pa[k], kk), pb[k]);
                }
                st_g(out + gi, o);
                Ot[rl * M + ej] = o;
              }
            }
          }
        }
        __syncthreads();
        // 2. layer r + 2 of the stage input is in flight while the Gram terms
        //    of layer r are formed; it replaces layer r - 1
        if (r + 2 < d_r) {
          const g_double2* nx = in + (size_t)(r + 2) * LM;
          double2 pf[kTPrefetch];
#pragma unroll
          for (int u = 0; u < kTPrefetch; ++u) {
            const int e = tid + u * kTW;
            if (e < LM) pf[u] = ld_g(nx + e);
          }
          add_terms(acc);
#pragma unroll
          for (int u = 0; u < kTPrefetch; ++u) {
            const int e = tid + u * kTW;
            if (e < LM) Yp[e] = pf[u];
          }
          for (int e = tid + kTPrefetch * kTW; e < LM; e += kTW) Yp[e] = ld_g(nx + e);
        } else {
          add_terms(acc);
        }
        __syncthreads();
        double2* t = Yp;
        Yp = Yc;
        Yc = Yn;
        Yn = t;
      }
      double f2 = 0.0;
      const bool last = (s == 3) && (n + 1 == nrun);
      const int rc = solve(acc, last, &f2);
      if (rc) {
        if (tid == 0) {
          report(T, rc, step);
          *T.step = step;
        }
        return;
      }
      if (last && tid == 0) *T.fro2 = f2;
    }
  }
  for (int e = tid; e < 2 * MM; e += kTW) st_g(gW + e, Wl[e]);
  if (tid == 0) *T.step = step0 + nrun;
}

// blockIdx.x = trajectory of trajs[]; the RK4 chunk and the prologue are
// separate kernels so that timing tools see the step kernel alone.
template <int KP>
__global__ __launch_bounds__(kTW) void k_packed(const TrajDev* __restrict__ trajs, int64_t step0, int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.mkind == 1) {
    if (T.frame)
      packed_body<KP, true, 1>(T, 0, step0, nchunk);
    else
      packed_body<KP, false, 1>(T, 0, step0, nchunk);
  } else if (T.frame)
    packed_body<KP, true>(T, 0, step0, nchunk);
  else
    packed_body<KP, false>(T, 0, step0, nchunk);
}
template <int KP>
__global__ __launch_bounds__(kTW) void k_packed_prologue(const TrajDev* __restrict__ trajs, int64_t step0,
                                                         int64_t nchunk) {
  packed_body<KP, false>(trajs[blockIdx.x], 1, step0, nchunk);
}

constexpr int kPackedKP[] = {2, 3, 5, 8, 12, 16};
template <int I = 0>
inline const void* packed_kernel(int kp, bool prologue) {
  if constexpr (I + 1 < (int)(sizeof(kPackedKP) / sizeof(int))) {
    if (kp > kPackedKP[I]) return packed_kernel<I + 1>(kp, prologue);
  }
  return prologue ? (const void*)k_packed_prologue<kPackedKP[I]> : (const void*)k_packed<kPackedKP[I]>;
}

}  // namespace lrk
