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

#include <type_traits>

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
// doubles) and sqrt(0 .. dmax), dmax = max(d_q, d_r, d_f).  The normal-mode
// model (kind 2) holds nine tiles (five input layers, the filter jump of two
// layers, the output of two) and stages its M x 4M Gram terms beside the
// elimination matrix.
__host__ __device__ inline size_t packed_lds_elems(int L, int M, int dmax, int kind = 0) {
  const size_t tiles = (kind == 2 ? 9 : 4) * (size_t)L * M, aug = (kind == 2 ? 7 : 3) * (size_t)M * M;
  // (+16: the Gram-term row blocks may read up to 15 elements past the output tile)
  return (tiles > aug ? tiles : aug) + 2 * (size_t)M * M + 10 * kTDriveWin + 3 * (size_t)M +
         (5 * (size_t)L + dmax + 2) / 2 + 16;
}
// Entries of the Gram terms per thread: thread t owns column t mod C (C = 3M
// columns [G | C_1 | C_2], or 4M for kind 2) and the block of KPe consecutive
// rows from (t / C) KPe, KPe = ceil(M / NG), NG = 256 / C row groups.  Kernel
// variants exist for a few block sizes KP >= KPe (the entries past KPe are
// computed and dropped).
__host__ __device__ inline int packed_kpe(int M, int C) {
  const int ng = kTW / C;
  return (M + ng - 1) / ng;
}
inline int packed_kp(int M, int kind = 0) {
  const int need = packed_kpe(M, (kind == 2 ? 4 : 3) * M);
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

// Kind 2: K rows of Q = O^ sqrt(kappa) c_l^ O over one layer pair, acc[k] +=
// c sum_rl conj(Ot[rl][pi0 + k]) Op[rl][pcc], Ot the output of layer r, Op that
// of layer r - 1 and c = sqrt(kappa r).
template <int K, int KP>
__device__ __forceinline__ void gram_rows_q(double2 (&acc)[KP], const double2* Ot, const double2* Op, double c,
                                            int L, int M, int pcc, int pi0) {
  for (int rl = 0; rl < L; ++rl) {
    const double2 x = cscale(c, Op[rl * M + pcc]);
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
  if (!P.pact || P.pkind > 2) return;
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

// Kind 2: the Q columns (pkind 3) of the layer pair (Ot, Op), c = sqrt(kappa r).
template <int KP>
__device__ __forceinline__ void packed_terms_q(double2 (&acc)[KP], const PackedMap& P, const double2* Ot,
                                               const double2* Op, double c) {
  if (!P.pact || P.pkind != 3) return;
  const int L = P.L, M = P.M, KPe = P.KPe, pcc = P.pcc, pi0 = P.pi0;
  if (KPe <= 2 || KP == 2) {
    gram_rows_q<2>(acc, Ot, Op, c, L, M, pcc, pi0);
  } else if (KPe <= 3 || KP == 3) {
    if constexpr (KP >= 3) gram_rows_q<3>(acc, Ot, Op, c, L, M, pcc, pi0);
  } else if (KPe <= 5 || KP == 5) {
    if constexpr (KP >= 5) gram_rows_q<5>(acc, Ot, Op, c, L, M, pcc, pi0);
  } else if (KPe <= 8 || KP == 8) {
    if constexpr (KP >= 8) gram_rows_q<8>(acc, Ot, Op, c, L, M, pcc, pi0);
  } else if (KPe <= 12 || KP == 12) {
    if constexpr (KP >= 12) gram_rows_q<12>(acc, Ot, Op, c, L, M, pcc, pi0);
  } else {
    if constexpr (KP >= 16) gram_rows_q<16>(acc, Ot, Op, c, L, M, pcc, pi0);
  }
}

// Gauss-Jordan elimination of the M x 3M matrix [G | C_1 | C_2] in Aug, then
// W_k = X_k^ into Wl (X_k the solved right-hand sides); returns 0 or -4 (pivot
// <= 0).  Thread t keeps column c = t mod 3M and the rows t / 3M, t / 3M + NG,
// ... (NG = 256 / 3M row groups).  Pivot p updates every entry right of the
// pivot column in the rows other than p, x - (Aug[i][p] / Aug[p][p]) Aug[p][c];
// the pivot row and the pivot column are only read while it runs, so one
// barrier per pivot suffices, and the rows are divided by their pivots at the
// end (a pivot row is not changed by later pivots left of its own column).
__device__ __forceinline__ int packed_eliminate(double2* Aug, double2* Wl, double2* /* unused */, int M) {
  const int tid = threadIdx.x, C3 = 3 * M, MM = M * M;
  const int ng = kTW / C3, c = tid % C3, g = tid / C3;
  const bool act = g < ng;
  for (int p = 0; p < M; ++p) {
    const double piv = Aug[p * C3 + p].x;
    if (!(piv > 0.0)) return -4;
    if (act && c > p) {
      const double rp = pivot_rcp(piv);
      const double2 pr = Aug[p * C3 + c];
      for (int i = g; i < M; i += ng) {
        if (i != p) {
          const double2 l = cscale(rp, Aug[i * C3 + p]);
          Aug[i * C3 + c] = cadd(Aug[i * C3 + c], cmul(make_double2(-l.x, -l.y), pr));
        }
      }
    }
    __syncthreads();
  }
  // W_k[i][j] = conj(X_k[j][i]), X_k[j] = row j of the columns M (k + 1) .. over its pivot
  for (int e = tid; e < 2 * MM; e += kTW) {
    const int k = e / MM, o = e - k * MM, i = o / M, j = o - i * M;
    const double2 x = cscale(pivot_rcp(Aug[j * C3 + j].x), Aug[j * C3 + M * (k + 1) + i]);
    Wl[e] = make_double2(x.x, -x.y);
  }
  __syncthreads();
  return 0;
}

// The threads' entries of the Gram terms into St (row stride P.C3), with the
// non-finite check and, on request, ||G||_F^2; returns 0 or -5.
template <int KP>
__device__ __forceinline__ int packed_store(double2 (&acc)[KP], const PackedMap& P, double2* St, double* s_red,
                                            int* s_flag, bool want_fro2, double* fro2) {
  const int tid = threadIdx.x, M = P.M, C = P.C3, KPe = P.KPe, pi0 = P.pi0, pc = P.pc;
  __syncthreads();  // the tiles are free
  int bad = 0;
  double f2 = 0.0;
  if (P.pact) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = pi0 + k;
      if (k < KPe && i < M) {
        St[i * C + pc] = acc[k];
        if (!isfinite(acc[k].x) || !isfinite(acc[k].y)) bad = 1;
        if (P.pkind == 0) f2 += acc[k].x * acc[k].x + acc[k].y * acc[k].y;
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
  return *s_flag ? -5 : 0;
}

// Kind 2: [G | P_u | C_2 | Q] (staged in St, M x 4M) -> [G | C_1 | C_2] in
// Aug, with P_u = sqrt(kappa) O^ c_u O and Q = sqrt(kappa) O^ c_l^ O:
// O^ L_1 O = e1 (s_21 P_u^ + s_22 Q) + conj(e1) (s_23 Q^ + s_24 P_u), e1 the
// frame phase e^{i w_d t} of the time the W_k are used at (1 in the lab frame).
__device__ __forceinline__ void packed_form_c1(const double2* St, double2* Aug, int M, const double* nm,
                                               double2 e1) {
  const int C3 = 3 * M, C4 = 4 * M;
  const double2 e1c = make_double2(e1.x, -e1.y);
  for (int e = threadIdx.x; e < M * C3; e += kTW) {
    const int i = e / C3, c = e - i * C3;
    double2 v;
    if (c < M || c >= 2 * M) {
      v = St[i * C4 + c];
    } else {
      const int j = c - M;
      const double2 pij = St[i * C4 + M + j], pji = St[j * C4 + M + i];
      const double2 qij = St[i * C4 + 3 * M + j], qji = St[j * C4 + 3 * M + i];
      // s_21 conj(P_u[j][i]) + s_22 Q[i][j] and s_23 conj(Q[j][i]) + s_24 P_u[i][j]
      const double2 cr = make_double2(nm[0] * pji.x + nm[1] * qij.x, -nm[0] * pji.y + nm[1] * qij.y);
      const double2 an = make_double2(nm[2] * qji.x + nm[3] * pij.x, -nm[2] * qji.y + nm[3] * pij.y);
      v = cadd(cmul(e1, cr), cmul(e1c, an));
    }
    Aug[e] = v;
  }
  __syncthreads();
}

// [G | C_1 | C_2] (the threads' entries) -> W_1, W_2 in Wl, through the M x 3M
// elimination in Aug; returns 0, or -4 (pivot <= 0) / -5 (non-finite).
template <int KP>
__device__ __forceinline__ int packed_solve(double2 (&acc)[KP], const PackedMap& P, double2* Aug, double2* Wl,
                                            double2* s_prow, double* s_red, int* s_flag, bool want_fro2,
                                            double* fro2) {
  const int rc = packed_store<KP>(acc, P, Aug, s_red, s_flag, want_fro2, fro2);
  return rc ? rc : packed_eliminate(Aug, Wl, s_prow, P.M);
}

// ---------------------------------------------------------------- Gram terms on the matrix cores
//
// The products [G | C_1 | C_2] += O^ [O | L_1 O | L_2 O] of one output layer O
// (L x M, in LDS) as 16 x 16 output tiles of v_mfma instructions.  Per chunk
// of layer rows an output tile (rows i = columns of O, columns c of
// [O | L_1 O | L_2 O]) gains
//   Re += A_re B_re + A_im B_im,   Im += A_re B_im - A_im B_re,
// A[i][k] = O[n0 + k][i], B[k][c] = [O | L_1 O | L_2 O][n0 + k][c]: four real
// products.  Arithmetic by mode:
//   0 FP64:   v_mfma_f64_16x16x4f64 (rows in chunks of 4);
//   1 FP32:   v_mfma_f32_16x16x4f32, operands rounded to FP32, FP32 accumulation;
//   2 BF16x3: C_k from the three leading products hi hi + hi lo + lo hi of the
//             BF16 parts of the FP32-rounded operands (v_mfma_f32_16x16x16_bf16,
//             rows in chunks of 16, FP32 accumulation); G in FP64 (as in the
//             spread schedule: the split products do not resolve the smallest
//             eigenvalues of G).
// Lane layouts: A[i][k] at lane i + 16 k and B[k][c] at lane c + 16 k (BF16:
// lane c + 16 (k / 4), element k mod 4); D[4 v + l / 16][l mod 16] for FP64
// and D[4 (l / 16) + v][l mod 16] for FP32 / BF16, v = 0..3, at lane l.
// Tiles: IT = ceil(M / 16) row tiles.  Modes 0 and 1 tile the 3M columns
// densely (tile t: row tile t mod IT, column tile t / IT, wave t mod 4, slot
// t / 4: two slots for M <= 21, three for M <= 32); mode 2 gives each of the IT^2 G tiles a
// wave and tiles [C_1 | C_2] per block (2 IT^2 tiles, two slots).  With IT
// dividing 4, every slot of a wave has the same row tile: A is loaded once
// per chunk.
typedef double mg_d4 __attribute__((ext_vector_type(4)));
typedef float mg_f4 __attribute__((ext_vector_type(4)));
typedef short mg_s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mg_d4 mg_mm(double a, double b, mg_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mg_f4 mg_mm(float a, float b, mg_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mg_f4 mg_mm(mg_s4 a, mg_s4 b, mg_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// BF16 parts of x rounded to FP32: x ~ hi + lo (bit patterns)
__device__ __forceinline__ void mg_split(double x, short& hi, short& lo) {
  const float f = (float)x;
  const float h = bf16_rne(f);
  hi = (short)(__float_as_uint(h) >> 16);
  lo = (short)(__float_as_uint(bf16_rne(f - h)) >> 16);
}
// the jump row of column block pk: coefficient and source row of row n of
// [O | L_1 O | L_2 O] (coef[0 .. L) = 1; 0 where the jump leaves the mode)
__device__ __forceinline__ double2 mg_bval(const double2* Ot, const double* coef, int L, int M, int d_f, int pk,
                                           int cc, int n) {
  const int sh = pk == 0 ? 0 : (pk == 1 ? 1 : d_f);
  return cscale(coef[pk * L + n], Ot[min(n + sh, L - 1) * M + cc]);
}

// Entry (i, pk M + cc) of [G | C_1 | C_2] into Aug (row stride 3M) with the
// non-finite check and ||G||_F^2.
__device__ __forceinline__ void mg_put(double2* Aug, int M, int i, int pk, int cc, double re, double im, int& bad,
                                       double& f2) {
  Aug[i * 3 * M + pk * M + cc] = make_double2(re, im);
  if (!isfinite(re) || !isfinite(im)) bad = 1;
  if (pk == 0) f2 += re * re + im * im;
}

// Flag and ||G||_F^2 of the stored entries across the workgroup; returns 0 or -5.
__device__ __forceinline__ int mg_finish(int bad, double f2, double* s_red, int* s_flag, bool want_fro2,
                                         double* fro2) {
  const int tid = threadIdx.x;
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
  return *s_flag ? -5 : 0;
}

// Modes 0 (FP64) and 1 (FP32), NS output tiles per wave.
template <int GP, int NS>
struct MGramDense {
  typedef typename std::conditional<GP == 0, mg_d4, mg_f4>::type Acc;
  typedef typename std::conditional<GP == 0, double, float>::type R;
  static constexpr int kMgSlots = NS;
  Acc re[kMgSlots], im[kMgSlots];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int u = 0; u < kMgSlots; ++u) re[u] = im[u] = Acc{0, 0, 0, 0};
  }
  __device__ __forceinline__ void add_layer(const double2* Ot, const double* coef, int L, int M, int d_f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int IT = (M + 15) >> 4, tot = IT * ((3 * M + 15) >> 4);
    const int acol = (w % IT) * 16 + li;  // column of O in the A operand (the same for every slot)
    int pk[kMgSlots], cc[kMgSlots];
    bool bv[kMgSlots];
#pragma unroll
    for (int u = 0; u < kMgSlots; ++u) {
      const int t = w + 4 * u, c = (t / IT) * 16 + li;
      pk[u] = c / M;
      cc[u] = c - pk[u] * M;
      bv[u] = t < tot && c < 3 * M;
    }
    for (int n0 = 0; n0 < L; n0 += 4) {
      const int n = n0 + lk;
      const double2 a = (n < L && acol < M) ? Ot[n * M + acol] : make_double2(0.0, 0.0);
      const R ar = (R)a.x, ai = (R)a.y, ain = -ai;
#pragma unroll
      for (int u = 0; u < kMgSlots; ++u) {
        if (w + 4 * u < tot) {  // uniform in the wave
          const double2 b = (n < L && bv[u]) ? mg_bval(Ot, coef, L, M, d_f, pk[u], cc[u], n) : make_double2(0.0, 0.0);
          const R br = (R)b.x, bi = (R)b.y;
          re[u] = mg_mm(ar, br, re[u]);
          re[u] = mg_mm(ai, bi, re[u]);
          im[u] = mg_mm(ar, bi, im[u]);
          im[u] = mg_mm(ain, br, im[u]);
        }
      }
    }
  }
  // the entries into Aug (M x 3M); returns 0 or -5
  __device__ __forceinline__ int store(double2* Aug, int M, double* s_red, int* s_flag, bool want_fro2,
                                       double* fro2) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int IT = (M + 15) >> 4, tot = IT * ((3 * M + 15) >> 4);
    __syncthreads();  // the tiles are free
    int bad = 0;
    double f2 = 0.0;
#pragma unroll
    for (int u = 0; u < kMgSlots; ++u) {
      const int t = w + 4 * u;
      if (t >= tot) continue;
      const int c = (t / IT) * 16 + li;
      if (c >= 3 * M) continue;
      const int pk = c / M, cc = c - pk * M;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (t % IT) * 16 + (GP == 0 ? 4 * v + lk : 4 * lk + v);
        if (i < M) mg_put(Aug, M, i, pk, cc, (double)re[u][v], (double)im[u][v], bad, f2);
      }
    }
    return mg_finish(bad, f2, s_red, s_flag, want_fro2, fro2);
  }
};

// Mode 2 (BF16x3 C_k, FP64 G).
struct MGramSplit {
  mg_d4 gre, gim;            // the wave's G tile
  mg_f4 cre[2], cim[2];      // its two C tiles

  __device__ __forceinline__ void zero() {
    gre = gim = mg_d4{0, 0, 0, 0};
    cre[0] = cre[1] = cim[0] = cim[1] = mg_f4{0, 0, 0, 0};
  }
  __device__ __forceinline__ void add_layer(const double2* Ot, const double* coef, int L, int M, int d_f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int IT = (M + 15) >> 4;
    const int acol = (w % IT) * 16 + li;
    // G tile w (row tile w mod IT, column tile w / IT): FP64, rows in chunks of 4
    if (w < IT * IT) {
      const int bcol = (w / IT) * 16 + li;
      for (int n0 = 0; n0 < L; n0 += 4) {
        const int n = n0 + lk;
        const double2 a = (n < L && acol < M) ? Ot[n * M + acol] : make_double2(0.0, 0.0);
        const double2 b = (n < L && bcol < M) ? Ot[n * M + bcol] : make_double2(0.0, 0.0);
        gre = mg_mm(a.x, b.x, gre);
        gre = mg_mm(a.y, b.y, gre);
        gim = mg_mm(a.x, b.y, gim);
        gim = mg_mm(-a.y, b.x, gim);
      }
    }
    // C tiles t = w, w + 4 of [C_1 | C_2] (row tile t mod IT, column tile t / IT of 2 IT): BF16x3,
    // rows in chunks of 16 (lane rows n0 + 4 lk + e)
    const int ntc = 2 * IT * IT;
    int pk[2], cc[2];
    bool bv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = w + 4 * u, ct = t / IT;
      pk[u] = 1 + ct / IT;
      cc[u] = (ct % IT) * 16 + li;
      bv[u] = t < ntc && cc[u] < M;
    }
    if (w >= ntc) return;
    for (int n0 = 0; n0 < L; n0 += 16) {
      mg_s4 arh, arl, aih, ail, ainh, ainl;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + 4 * lk + e;
        const double2 a = (n < L && acol < M) ? Ot[n * M + acol] : make_double2(0.0, 0.0);
        short h, l;
        mg_split(a.x, h, l);
        arh[e] = h;
        arl[e] = l;
        mg_split(a.y, h, l);
        aih[e] = h;
        ail[e] = l;
        ainh[e] = (short)(h ^ (short)0x8000);  // -a_im: the sign bit of each part
        ainl[e] = (short)(l ^ (short)0x8000);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (w + 4 * u < ntc) {  // uniform in the wave
          mg_s4 brh, brl, bih, bil;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int n = n0 + 4 * lk + e;
            const double2 b =
                (n < L && bv[u]) ? mg_bval(Ot, coef, L, M, d_f, pk[u], cc[u], n) : make_double2(0.0, 0.0);
            short h, l;
            mg_split(b.x, h, l);
            brh[e] = h;
            brl[e] = l;
            mg_split(b.y, h, l);
            bih[e] = h;
            bil[e] = l;
          }
          // each real product from its three leading part products (smallest first)
          cre[u] = mg_mm(arl, brh, cre[u]);
          cre[u] = mg_mm(arh, brl, cre[u]);
          cre[u] = mg_mm(arh, brh, cre[u]);
          cre[u] = mg_mm(ail, bih, cre[u]);
          cre[u] = mg_mm(aih, bil, cre[u]);
          cre[u] = mg_mm(aih, bih, cre[u]);
          cim[u] = mg_mm(arl, bih, cim[u]);
          cim[u] = mg_mm(arh, bil, cim[u]);
          cim[u] = mg_mm(arh, bih, cim[u]);
          cim[u] = mg_mm(ainl, brh, cim[u]);
          cim[u] = mg_mm(ainh, brl, cim[u]);
          cim[u] = mg_mm(ainh, brh, cim[u]);
        }
      }
    }
  }
  __device__ __forceinline__ int store(double2* Aug, int M, double* s_red, int* s_flag, bool want_fro2,
                                       double* fro2) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int IT = (M + 15) >> 4;
    __syncthreads();  // the tiles are free
    int bad = 0;
    double f2 = 0.0;
    if (w < IT * IT) {
      const int j = (w / IT) * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (w % IT) * 16 + 4 * v + lk;
        if (i < M && j < M) mg_put(Aug, M, i, 0, j, gre[v], gim[v], bad, f2);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = w + 4 * u, ct = t / IT;
      if (t >= 2 * IT * IT) continue;
      const int pk = 1 + ct / IT, cc = (ct % IT) * 16 + li;
      if (cc >= M) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (t % IT) * 16 + 4 * lk + v;
        if (i < M) mg_put(Aug, M, i, pk, cc, (double)cre[u][v], (double)cim[u][v], bad, f2);
      }
    }
    return mg_finish(bad, f2, s_red, s_flag, want_fro2, fro2);
  }
};

template <int GM, int NS>
struct MGramOf {
  typedef MGramDense<GM, NS> type;
};
template <int NS>
struct MGramOf<2, NS> {
  typedef MGramSplit type;
};
// Output tiles per wave of the dense modes for rank M.
__host__ __device__ inline int mg_slots(int M) {
  const int it = (M + 15) / 16;
  return (it * ((3 * M + 15) / 16) + 3) / 4;
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

// Element (rl, j) of layer r for the normal-mode model (kind 2): z = H_eff Y with
// H_eff = diag(E_q + w_l r + w_u f) + i g n_t (mu_l (c_l^ - c_l) + mu_u (c_u^ -
// c_u)) + d(t) i (nu_l (c_l^ - c_l) + nu_u (c_u^ - c_u)) - i/2 (gamma b^b +
// L_1^ L_1).  The diagonal of L_1^ L_1 (the products of the truncated ladders:
// c c^ is n + 1 below the top level and 0 on it) is in hd (row part) and him
// (layer part); its off-diagonal part, kappa times
//   (s21 s22 + s23 s24)(c_l^ c_u + c_u^ c_l)
//   + (s22 s23 c_l^2 + (s21 s23 + s22 s24) c_l c_u + s21 s24 c_u^2) e^{-2 i w_d t}
//   + (the adjoint terms, raising twice) e^{2 i w_d t},
// reaches two layers up and down (Y[0..4] = layers r - 2 .. r + 2).  Phases as
// in packed_stencil_tm: a tap from a neighbour with dn more excitations
// carries e^{-i w_d t dn} in the rotating frame.
template <bool ROT>
__device__ __forceinline__ double2 packed_stencil_nm(const TrajDev& T, const double2* const* Y, const double* sq,
                                                     const double2* hd, const double* nt, const double2* ph,
                                                     int ph0, int r, int rl, int q, int f, int j, double drv,
                                                     double him) {
  const int M = T.M, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const double2 *Ym2 = Y[0], *Ym1 = Y[1], *Y0 = Y[2], *Yp1 = Y[3], *Yp2 = Y[4];
  const double s21 = T.nm[0], s22 = T.nm[1], s23 = T.nm[2], s24 = T.nm[3];
  const double mu_l = T.nm[4], mu_u = T.nm[5], nu_l = T.nm[6], nu_u = T.nm[7];
  const double2 h = hd[rl];
  double2 z = cmul(make_double2(h.x + T.w_r * r, h.y + him), Y0[rl * M + j]);
  const double sr0 = sq[r], sr1 = sq[min(r + 1, d_r)], sf0 = sq[f], sf1 = sq[min(f + 1, d_f)];
  const bool rdn = r > 0, rup = r + 1 < d_r, fdn = f > 0, fup = f + 1 < d_f;
  auto tap = [&](double2 acc, double c, int dn, double2 nb) {
    if (!ROT || dn == 0) return cfma(c, nb, acc);
    const double2 e = ph[dn + ph0];
    return cadd(acc, cmul(make_double2(c * e.x, -c * e.y), nb));
  };
  // i g n_t (mu_l (c_l^ - c_l) + mu_u (c_u^ - c_u))
  double2 s = make_double2(0.0, 0.0);
  for (int p = 0; p < d_q; ++p) {
    const double c = nt[q * d_q + p];
    if (c == 0.0) continue;
    const int row = p * d_f + f;
    if (rdn) s = tap(s, c * mu_l * sr0, p - q - 1, Ym1[row * M + j]);
    if (rup) s = tap(s, -c * mu_l * sr1, p - q + 1, Yp1[row * M + j]);
    if (fdn) s = tap(s, c * mu_u * sf0, p - q - 1, Y0[(row - 1) * M + j]);
    if (fup) s = tap(s, -c * mu_u * sf1, p - q + 1, Y0[(row + 1) * M + j]);
  }
  z = make_double2(z.x - T.g * s.y, z.y + T.g * s.x);
  // d(t) i (nu_l (c_l^ - c_l) + nu_u (c_u^ - c_u))
  double2 v = make_double2(0.0, 0.0);
  if (rdn) v = tap(v, nu_l * sr0, -1, Ym1[rl * M + j]);
  if (rup) v = tap(v, -nu_l * sr1, 1, Yp1[rl * M + j]);
  if (fdn) v = tap(v, nu_u * sf0, -1, Y0[(rl - 1) * M + j]);
  if (fup) v = tap(v, -nu_u * sf1, 1, Y0[(rl + 1) * M + j]);
  z = make_double2(z.x - drv * v.y, z.y + drv * v.x);
  // -i/2 kappa (off-diagonal part of f^ f)
  const double cx = s21 * s22 + s23 * s24, cb = s21 * s23 + s22 * s24, cl2 = s22 * s23, cu2 = s21 * s24;
  double2 w = make_double2(0.0, 0.0);
  if (rdn && fup) w = tap(w, cx * sr0 * sf1, 0, Ym1[(rl + 1) * M + j]);   // c_l^ c_u
  if (rup && fdn) w = tap(w, cx * sr1 * sf0, 0, Yp1[(rl - 1) * M + j]);   // c_u^ c_l
  if (r + 2 < d_r) w = tap(w, cl2 * sr1 * sq[r + 2], 2, Yp2[rl * M + j]);           // c_l c_l
  if (rup && fup) w = tap(w, cb * sr1 * sf1, 2, Yp1[(rl + 1) * M + j]);            // c_l c_u
  if (f + 2 < d_f) w = tap(w, cu2 * sf1 * sq[f + 2], 2, Y0[(rl + 2) * M + j]);      // c_u c_u
  if (r >= 2) w = tap(w, cl2 * sr0 * sq[r - 1], -2, Ym2[rl * M + j]);               // c_l^ c_l^
  if (rdn && fdn) w = tap(w, cb * sr0 * sf0, -2, Ym1[(rl - 1) * M + j]);           // c_l^ c_u^
  if (f >= 2) w = tap(w, cu2 * sf0 * sq[f - 1], -2, Y0[(rl - 2) * M + j]);          // c_u^ c_u^
  const double hk = 0.5 * T.kappa;
  return make_double2(z.x + hk * w.y, z.y - hk * w.x);
}

// Kind 2: element (rl, j) of L_1 Y at layer r, L_1 = sqrt(kappa) (s21 e1 c_u^ +
// s22 e1 c_l^ + s23 conj(e1) c_l + s24 conj(e1) c_u), from the layers r - 1,
// r, r + 1 (e1 = e^{i w_d t} in the rotating frame, 1 in the lab frame).
__device__ __forceinline__ double2 packed_jump_nm(const TrajDev& T, const double2* Ym1, const double2* Y0,
                                                  const double2* Yp1, const double* sq, int r, int rl, int f, int j,
                                                  double2 e1) {
  const int M = T.M, d_f = T.d_f, d_r = T.d_r;
  double2 up = make_double2(0.0, 0.0), dn = make_double2(0.0, 0.0);
  if (f > 0) up = cfma(T.nm[0] * sq[f], Y0[(rl - 1) * M + j], up);
  if (r > 0) up = cfma(T.nm[1] * sq[r], Ym1[rl * M + j], up);
  if (r + 1 < d_r) dn = cfma(T.nm[2] * sq[r + 1], Yp1[rl * M + j], dn);
  if (f + 1 < d_f) dn = cfma(T.nm[3] * sq[f + 1], Y0[(rl + 1) * M + j], dn);
  const double sk = sqrt(T.kappa);
  return cscale(sk, cadd(cmul(e1, up), cmulc(dn, e1)));
}

// ---------------------------------------------------------------- layer-split trajectories
//
// A trajectory can also be split over P workgroups ("parts") of one
// cooperative launch, for latency when few trajectories are in flight: part w
// owns the layers [w d_r / P, (w + 1) d_r / P) and runs the packed layer loop
// over them, reading its neighbour layers of the stage input from global
// memory.  After each pass the parts' Gram terms are summed (partials, group
// barrier A, a 1/P slice of the entries reduced in fixed order, group barrier
// B, the reduced entries back into every thread's registers), so that every
// part holds the same terms and solves the same M x M system.  Kind 2 pairs
// each layer with the one below it in the term Q: a part adds the pair across
// its upper boundary once the part above has published its first output
// layer (a point-to-point flag C).  Every buffer that another part reads goes
// through agent-coherent accesses; every wait is bounded as in the spread
// schedule.

// Part w's layer range.
__device__ __forceinline__ int split_lo(int w, int P, int d_r) { return (int)(((int64_t)w * d_r) / P); }
// Entries of the Gram terms a part publishes (M x 3M; kind 2: M x 4M).
__host__ __device__ inline int split_npe(int M, int kind) { return M * (kind == 2 ? 4 : 3) * M; }

// Layers r0 .. r0 + NL - 1 of a stage state in global memory into the LDS tiles dst[0 .. NL) (layers
// outside [0, d_r) are skipped), through agent-coherent loads that are all in flight before the
// first LDS store of a block (the loads of another part's layers are round trips through memory).
template <int NL>
__device__ __forceinline__ void split_load_layers(double2* const (&dst)[NL], const g_double2* src, int r0,
                                                  int d_r, int LM) {
  for (int e0 = 0; e0 < LM; e0 += 2 * kTW) {
    double2 v[NL][2];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = r0 + l, e = e0 + (int)threadIdx.x + u * kTW;
        v[l][u] = (r >= 0 && r < d_r && e < LM) ? ld_ag(src + (size_t)r * LM + e) : make_double2(0.0, 0.0);
      }
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = r0 + l, e = e0 + (int)threadIdx.x + u * kTW;
        if (r >= 0 && r < d_r && e < LM) dst[l][e] = v[l][u];
      }
  }
}

// Wait until one flag reaches target (bounded; raises the group's abort flag
// when the wait expires).
__device__ __forceinline__ bool flag_wait_one(const TrajDev& T, const g_u32* flag, uint32_t target, int* s_ok) {
  g_u32* abort_flag = (g_u32*)T.abort_flag;
  const uint32_t limit = T.spin_limit ? T.spin_limit : kSpinLimit;
  target += T.wait_bias;
  if (threadIdx.x == 0) {
    bool ok = true;
    uint32_t n = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++n > limit) {
        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *s_ok = ok ? 1 : 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return *s_ok != 0;
}

// Barrier counters of a part within one launch (the flags are zeroed before
// every launch; all parts pass the same barriers in the same order).
struct SplitSync {
  int w;
  uint32_t a, b, c;
};

// Sum of the parts' Gram terms (entry (i, c) of the M x C terms at i C + c)
// into the registers of every part; false when a group wait expired.
template <int KP>
__device__ bool split_sum(const TrajDev& T, double2 (&acc)[KP], const PackedMap& P, SplitSync& S, int* s_ok) {
  const int tid = threadIdx.x, C = P.C3, npe = P.M * C, np = T.P;
  g_double2* part = (g_double2*)T.PART;
  g_double2* red = (g_double2*)T.RED;
  if (P.pact) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = P.pi0 + k;
      if (k < P.KPe && i < P.M) st_ag(part + (size_t)S.w * npe + i * C + P.pc, acc[k]);
    }
  }
  g_u32* fA = (g_u32*)T.flagA;
  g_u32* fB = (g_u32*)T.flagB;
  flag_arrive(fA + (size_t)S.w * kFlagStride, ++S.a);
  if (!flag_wait(T, fA, S.a, s_ok)) return false;
  // slice of the entries: a group of G lanes per entry (G = 1 .. 16, the
  // smallest power of two with at most 8 parts per lane, else 16), lane l adds
  // the parts l, l + G, ... in order with up to 8 loads in flight, then a
  // butterfly over the group; the order depends on P only
  const int cs = (npe + np - 1) / np, e0 = S.w * cs, e1 = min(npe, e0 + cs);
  int G = 1;
  while (G < 16 && np > 8 * G) G <<= 1;
  const int sub = tid & (G - 1), grp = tid / G;
  for (int e = e0 + grp; e < e1; e += kTW / G) {
    double2 s = make_double2(0.0, 0.0);
    for (int q0 = sub; q0 < np; q0 += 8 * G) {
      double2 pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * G;
        pv[u] = q < np ? ld_ag(part + (size_t)q * npe + e) : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u * G < np) s = cadd(s, pv[u]);
    }
    for (int off = G / 2; off > 0; off >>= 1) {
      s.x += __shfl_xor(s.x, off, G);
      s.y += __shfl_xor(s.y, off, G);
    }
    if (sub == 0) st_ag(red + e, s);
  }
  flag_arrive(fB + (size_t)S.w * kFlagStride, ++S.b);
  if (!flag_wait(T, fB, S.b, s_ok)) return false;
  if (P.pact) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = P.pi0 + k;
      acc[k] = (k < P.KPe && i < P.M) ? ld_ag(red + i * C + P.pc) : make_double2(0.0, 0.0);
    }
  }
  return true;
}

// Sum of one value per part, the same in every part (parts in order); false
// when the group wait expired.
__device__ bool split_sum_value(const TrajDev& T, double v, double* out, SplitSync& S, int* s_ok) {
  g_double* vals = (g_double*)(T.RED + T.npe);
  if (threadIdx.x == 0) __hip_atomic_store(vals + S.w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  g_u32* fA = (g_u32*)T.flagA;
  flag_arrive(fA + (size_t)S.w * kFlagStride, ++S.a);
  if (!flag_wait(T, fA, S.a, s_ok)) return false;
  double tot = 0.0;
  for (int q = 0; q < T.P; ++q) tot += __hip_atomic_load(vals + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *out = tot;
  return true;
}

// Kind 2: publish the first output layer of the pass (flag C of the part).
__device__ __forceinline__ void split_publish_first(const TrajDev& T, SplitSync& S) {
  g_u32* fC = (g_u32*)T.flagB + (size_t)T.P * kFlagStride;
  flag_arrive(fC + (size_t)S.w * kFlagStride, S.c);
}
// Kind 2: wait for the first output layer of the part above.
__device__ __forceinline__ bool split_wait_above(const TrajDev& T, const SplitSync& S, int* s_ok) {
  const g_u32* fC = (const g_u32*)T.flagB + (size_t)T.P * kFlagStride;
  return flag_wait_one(T, fC + (size_t)(S.w + 1) * kFlagStride, S.c, s_ok);
}

// The kernel body: prologue (Gram terms and W of the initial state, no step)
// or a chunk of nchunk RK4 steps from step0.  KP = entries of the Gram terms
// per thread (packed_kp).  MK = model kind; kind 2 keeps five input layers,
// the filter jump L_1 Y of the current and the next layer, and the outputs of
// the current and the previous layer (for the cross-layer term Q).
template <int KP, bool ROT, int MK = 0, int GM = -1, int NS = 2, bool SPLIT = false>
__device__ __forceinline__ void packed_body(const TrajDev& T, int prologue, int64_t step0, int64_t nchunk,
                                            int part = 0) {
  extern __shared__ double2 lds[];
  __shared__ double s_red[kTW / 64];
  __shared__ double s_nt[kMaxDq * kMaxDq];
  __shared__ double2 s_ph[2 * kMaxDq + 3];  // e^{i w_d t m}, m = -(d_q + 1) .. d_q + 1, of the stage (kinds 1, 2, rotating frame)
  __shared__ int s_flag;
  __shared__ int s_ok;
  constexpr bool NM = MK == 2;
  constexpr int NTILE = NM ? 9 : 4;
  const int tid = threadIdx.x;
  const int M = T.M, MM = M * M, L = T.L, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const int LM = L * M, CT = (NM ? 4 : 3) * M;
  const double dt = T.dt;
  const double sk = sqrt(T.kappa), sg = sqrt(T.gamma);
  double2* Ym2 = lds;                                 // kind 2: layer r - 2 of the stage input
  double2* Yp = lds;                                  // layers r - 1, r, r + 1 of the stage input
  double2* Yc = lds + LM;
  double2* Yn = lds + 2 * LM;
  double2* Yp2 = lds;                                 // kind 2: layer r + 2
  double2* Y1c = lds + 5 * LM;                        // kind 2: L_1 Y of layers r, r + 1
  double2* Y1n = lds + 6 * LM;
  double2* Ot = lds + (NM ? 7 : 3) * LM;              // layer r of the stage output
  double2* Op = lds + 8 * LM;                         // kind 2: layer r - 1 of the stage output
  const int areg = (NM ? 7 : 3) * MM;
  double2* St = lds;                                  // Gram terms as formed (M x CT)
  double2* Aug = NM ? lds + 4 * MM : lds;             // M x 3M elimination (after the layer loop)
  double2* Wl = lds + (NTILE * LM > areg ? NTILE * LM : areg);  // W_1, W_2 (M x M each, row i, column j)
  double (*s_dtab)[5] = reinterpret_cast<double (*)[5]>(Wl + 2 * MM);  // [4 kTDriveWin][5] drive table
  double2* s_prow = Wl + 2 * MM + 10 * kTDriveWin;          // [3M] pivot row
  double2* hd = s_prow + 3 * M;                             // [L] diagonal of H_eff without its layer term
  double* coef = reinterpret_cast<double*>(hd + L);         // [3][L]: 1, filter jump, transmon jump
  double* sq = coef + 3 * L;                                // sqrt(0 .. dmax)
  g_double2* gBb = (g_double2*)T.Bb;
  g_double2* gacc = (g_double2*)T.acc;
  g_double2* gW = (g_double2*)T.W;

  if (tid == 0) s_flag = *T.status;
  if constexpr (MK >= 1)
    for (int i = tid; i < d_q * d_q; i += kTW) s_nt[i] = T.ntq[i];
  for (int rl = tid; rl < L; rl += kTW) {
    const int q = rl / d_f, f = rl - q * d_f;
    const double eq = MK >= 1 ? T.Et[q] - (ROT ? T.w_d * q : 0.0) : T.w_q * q + 0.5 * T.alpha * q * (q - 1);
    // kind 2: the f-dependent diagonal of f^ f, s21^2 c_u c_u^ + s24^2 c_u^ c_u
    const double ff = NM ? T.nm[0] * T.nm[0] * (f + 1 < d_f ? f + 1.0 : 0.0) + T.nm[3] * T.nm[3] * f : (double)f;
    hd[rl] = make_double2(eq + T.w_f * f, -0.5 * (T.kappa * ff + T.gamma * q));
    coef[rl] = 1.0;
    coef[L + rl] = (f + 1 < d_f) ? sk * sqrt((double)(f + 1)) : 0.0;
    coef[2 * L + rl] = (q + 1 < d_q) ? sg * sqrt((double)(q + 1)) : 0.0;
  }
  for (int k = tid; k <= max(max(d_q, d_r), d_f); k += kTW) sq[k] = sqrt((double)k);
  __syncthreads();
  if (s_flag != 0) return;
  const int64_t nrun = prologue ? 0 : (step0 < T.nsteps ? min(nchunk, T.nsteps - step0) : 0);
  if (!prologue && nrun <= 0) return;
  // layers of this workgroup: all of them, or those of its part of a split trajectory
  const int r_lo = SPLIT ? split_lo(part, T.P, d_r) : 0;
  const int r_hi = SPLIT ? split_lo(part + 1, T.P, d_r) : d_r;
  SplitSync SS{part, 0u, 0u, 0u};
  auto ldS = [](const g_double2* p) -> double2 {
    if constexpr (SPLIT) return ld_ag(p);
    else return ld_g(p);
  };
  auto stS = [](g_double2* p, double2 v) {
    if constexpr (SPLIT) st_ag(p, v);
    else st_g(p, v);
  };

  // element mapping: column j, rows g, g + NGe, ...
  const int NGe = kTW / M;
  const int ej = tid % M, eg = tid / M;
  const bool eact = eg < NGe;
  // Gram-term mapping: column c of [O | L_1 O | L_2 O] (kind 2: [O | c_u O | L_2 O | c_l^ O]), rows i = pi0 + k
  const int NGp = kTW / CT, KPe = packed_kpe(M, CT);
  const int pc = tid % CT, pg = tid / CT, pi0 = pg * KPe;
  const bool pact = pg < NGp && pi0 < M;
  const int pkind = pc / M, pcc = pc - pkind * M;  // 0: G, 1: C_1 (filter), 2: C_2 (transmon), 3: Q (kind 2)

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

  const PackedMap PM{M, CT, L, d_f, KPe, pc, pi0, pkind, pcc, pact};
  // the Gram terms: entries held by the threads (vector ALU, GM < 0) or
  // output tiles of the matrix cores (GM = arithmetic mode of MGramDense /
  // MGramSplit)
  double2 acc[KP];
  typename MGramOf<(GM < 0 ? 0 : GM), NS>::type mg;
  auto zero_terms = [&]() {
    if constexpr (GM >= 0) {
      mg.zero();
    } else {
#pragma unroll
      for (int k = 0; k < KP; ++k) acc[k] = make_double2(0.0, 0.0);
    }
  };
  // Gram terms of the output layer r in Ot (kind 2: and of the pair (Op, Ot))
  auto add_terms = [&](int r) {
    if constexpr (GM >= 0) {
      mg.add_layer(Ot, coef, L, M, d_f);
    } else {
      packed_terms<KP>(acc, PM, Ot, coef);
      if constexpr (NM)
        if (r > r_lo) packed_terms_q<KP>(acc, PM, Ot, Op, sk * sq[r]);
    }
  };
  // W_k of the state whose Gram terms the threads hold, for use at time t_use
  auto solve = [&](bool want_fro2, double* fro2, double t_use) -> int {
    if constexpr (GM >= 0) {
      const int rc = mg.store(Aug, M, s_red, &s_flag, want_fro2, fro2);
      return rc ? rc : packed_eliminate(Aug, Wl, s_prow, M);
    } else if constexpr (NM) {
      const int rc = packed_store<KP>(acc, PM, St, s_red, &s_flag, want_fro2, fro2);
      if (rc) return rc;
      packed_form_c1(St, Aug, M, T.nm, ROT ? frame_phase(T.w_d, t_use) : make_double2(1.0, 0.0));
      return packed_eliminate(Aug, Wl, s_prow, M);
    } else {
      return packed_solve<KP>(acc, PM, Aug, Wl, s_prow, s_red, &s_flag, want_fro2, fro2);
    }
  };
  // kind 2: L_1 Y of layer r into dst from the layers r - 1, r, r + 1
  auto jump_tile = [&](double2* dst, const double2* ym, const double2* y0, const double2* yp, int r, double2 e1j) {
    for (int e = tid; e < LM; e += kTW) {
      const int rl = e / M, j = e - rl * M;
      dst[e] = packed_jump_nm(T, ym, y0, yp, sq, r, rl, rl % d_f, j, e1j);
    }
  };

  if (!SPLIT && prologue) {
    zero_terms();
    for (int r = 0; r < d_r; ++r) {
      __syncthreads();
      for (int e = tid; e < LM; e += kTW) Ot[e] = ld_g(gBb + (size_t)r * LM + e);
      __syncthreads();
      add_terms(r);
      if constexpr (NM) {
        double2* t = Ot;
        Ot = Op;
        Op = t;
      }
    }
    double f2 = 0.0;
    const int rc = solve(true, &f2, stage_time(step0, 0));
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
      const double2 e1j = ROT ? e1 : make_double2(1.0, 0.0);  // phase of the kind-2 filter jump
      zero_terms();
      if constexpr (MK >= 1 && ROT)
        if (tid < 2 * d_q + 3) s_ph[tid] = frame_phase((tid - d_q - 1) * T.w_d, stage_time(step, s));
      __syncthreads();  // Wl of this stage written; tiles free
      if constexpr (NM) {
        Ym2 = lds;
        Yp = lds + LM;
        Yc = lds + 2 * LM;
        Yn = lds + 3 * LM;
        Yp2 = lds + 4 * LM;
        Y1c = lds + 5 * LM;
        Y1n = lds + 6 * LM;
        Ot = lds + 7 * LM;
        Op = lds + 8 * LM;
      } else {
        Yp = lds;
        Yc = lds + LM;
        Yn = lds + 2 * LM;
      }
      if constexpr (SPLIT) {  // the window around the part's first layer, all loads in flight together
        if constexpr (NM) {
          double2* const w5[5] = {Ym2, Yp, Yc, Yn, Yp2};
          split_load_layers<5>(w5, in, r_lo - 2, d_r, LM);
        } else {
          double2* const w3[3] = {Yp, Yc, Yn};
          split_load_layers<3>(w3, in, r_lo - 1, d_r, LM);
        }
      } else {
        for (int e = tid; e < LM; e += kTW) Yc[e] = ld_g(in + e);
        if (d_r > 1)
          for (int e = tid; e < LM; e += kTW) Yn[e] = ld_g(in + LM + e);
        if constexpr (NM)
          if (d_r > 2)
            for (int e = tid; e < LM; e += kTW) Yp2[e] = ld_g(in + 2 * LM + e);
      }
      if constexpr (NM) {
        __syncthreads();
        jump_tile(Y1c, Yp, Yc, Yn, r_lo, e1j);
      }
      if constexpr (SPLIT) ++SS.c;
      __syncthreads();
      for (int r = r_lo; r < r_hi; ++r) {
        const double him = NM ? -0.5 * T.kappa *
                                    (T.nm[1] * T.nm[1] * (r + 1 < d_r ? r + 1.0 : 0.0) + T.nm[2] * T.nm[2] * r)
                              : 0.0;
        // 1. stage output of layer r, in blocks of kTRowBlock rows per thread
        if (eact) {
          const double2* A1 = NM ? Y1c : Yc;  // source tile of the filter jump rows
          for (int rb = eg; rb < L; rb += kTRowBlock * NGe) {
            // B_n and the RK4 accumulator of the block are in flight during the jump assembly
            double2 pb[kTRowBlock], pa[kTRowBlock];
            if (s > 0) {
#pragma unroll
              for (int k = 0; k < kTRowBlock; ++k) {
                const int rl = min(rb + k * NGe, L - 1);
                const size_t gi = ((size_t)r * L + rl) * M + ej;
                pb[k] = ldS(gBb + gi);
                pa[k] = ld_g(gacc + gi);  // the accumulator rows are the part's own
              }
            }
            double2 a1[kTRowBlock], a2[kTRowBlock];
            int s1[kTRowBlock], s2[kTRowBlock];  // source rows of the jumps, clamped into the tile
#pragma unroll
            for (int k = 0; k < kTRowBlock; ++k) {
              a1[k] = a2[k] = make_double2(0.0, 0.0);
              const int rl = min(rb + k * NGe, L - 1);
              s1[k] = (NM ? rl : min(rl + 1, L - 1)) * M;
              s2[k] = min(rl + d_f, L - 1) * M;
            }
            for (int i = 0; i < M; ++i) {
              const double2 w1 = Wl[i * M + ej], w2 = Wl[MM + i * M + ej];
#pragma unroll
              for (int k = 0; k < kTRowBlock; ++k) {
                a1[k] = cmac(a1[k], A1[s1[k] + i], w1);
                a2[k] = cmac(a2[k], Yc[s2[k] + i], w2);
              }
            }
#pragma unroll
            for (int k = 0; k < kTRowBlock; ++k) {
              const int rl = rb + k * NGe;
              if (rl < L) {
                const int q = rl / d_f, f = rl - q * d_f;
                const double2 a = cfma(NM ? 1.0 : coef[L + rl], a1[k], cscale(coef[2 * L + rl], a2[k]));
                double2 z;
                if constexpr (MK == 2) {
                  const double2* Yw[5] = {Ym2, Yp, Yc, Yn, Yp2};
                  z = packed_stencil_nm<ROT>(T, Yw, sq, hd, s_nt, s_ph, d_q + 1, r, rl, q, f, ej, drv, him);
                } else if constexpr (MK == 1) {
                  z = packed_stencil_tm<ROT>(T, Yp, Yc, Yn, sq, hd, s_nt, s_ph, d_q + 1, r, rl, q, f, ej, drv);
                } else {
                  z = packed_stencil<ROT>(T, Yp, Yc, Yn, sq, hd, r, rl, q, f, ej, drv, e1, e2);
                }
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
                stS(out + gi, o);
                Ot[rl * M + ej] = o;
              }
            }
          }
        }
        __syncthreads();
        if constexpr (SPLIT && NM)
          if (r == r_lo) split_publish_first(T, SS);
        // 2. the next input layer (r + 2; kind 2: r + 3) is in flight while the
        //    Gram terms of layer r are formed; it replaces the oldest layer
        const int rnx = NM ? r + 3 : r + 2;
        double2* dstl = NM ? Ym2 : Yp;
        if (rnx < (SPLIT ? min(d_r, r_hi + (NM ? 2 : 1)) : d_r)) {
          const g_double2* nx = in + (size_t)rnx * LM;
          double2 pf[kTPrefetch];
#pragma unroll
          for (int u = 0; u < kTPrefetch; ++u) {
            const int e = tid + u * kTW;
            if (e < LM) pf[u] = ldS(nx + e);
          }
          if constexpr (NM)
            if (r + 1 < r_hi) jump_tile(Y1n, Yc, Yn, Yp2, r + 1, e1j);
          add_terms(r);
#pragma unroll
          for (int u = 0; u < kTPrefetch; ++u) {
            const int e = tid + u * kTW;
            if (e < LM) dstl[e] = pf[u];
          }
          for (int e = tid + kTPrefetch * kTW; e < LM; e += kTW) dstl[e] = ldS(nx + e);
        } else {
          if constexpr (NM)
            if (r + 1 < r_hi) jump_tile(Y1n, Yc, Yn, Yp2, r + 1, e1j);
          add_terms(r);
        }
        __syncthreads();
        if constexpr (NM) {
          double2* t = Ym2;
          Ym2 = Yp;
          Yp = Yc;
          Yc = Yn;
          Yn = Yp2;
          Yp2 = t;
          t = Y1c;
          Y1c = Y1n;
          Y1n = t;
          t = Ot;
          Ot = Op;
          Op = t;
        } else {
          double2* t = Yp;
          Yp = Yc;
          Yc = Yn;
          Yn = t;
        }
      }
      if constexpr (SPLIT) {
        bool ok = true;
        if constexpr (NM) {
          if (r_hi < d_r) {  // the pair (r_hi - 1, r_hi) across the upper boundary
            ok = split_wait_above(T, SS, &s_ok);
            if (ok) {
              double2* const w1[1] = {Ot};
              split_load_layers<1>(w1, out, r_hi, d_r, LM);
              __syncthreads();
              packed_terms_q<KP>(acc, PM, Ot, Op, sk * sq[r_hi]);
            }
          }
        }
        if (ok) ok = split_sum<KP>(T, acc, PM, SS, &s_ok);
        if (!ok) {
          if (tid == 0) report(T, -8 /* LR_ERR_TIMEOUT */, step);
          return;
        }
      }
      double f2 = 0.0;
      const bool last = (s == 3) && (n + 1 == nrun);
      const int rc = solve(last, &f2, s < 3 ? stage_time(step, s + 1) : stage_time(step + 1, 0));
      if (rc) {
        if (tid == 0) {
          report(T, rc, step);
          *T.step = step;
        }
        return;
      }
      if (last && tid == 0 && (!SPLIT || part == 0)) *T.fro2 = f2;
    }
  }
  if (!SPLIT || part == 0) {
    for (int e = tid; e < 2 * MM; e += kTW) st_g(gW + e, Wl[e]);
    if (tid == 0) *T.step = step0 + nrun;
  }
}

// blockIdx.x = trajectory of trajs[]; the RK4 chunk and the prologue are
// separate kernels so that timing tools see the step kernel alone.  The
// normal-mode model has kernels of its own (its larger window would raise the
// register allocation, and so lower the occupancy, of the other kinds); up to
// entry blocks of 8 (M <= 21) they are held to two workgroups per CU, which
// spills ~30 VGPRs to scratch and measured 1.9x faster at the paper's size
// than one workgroup per CU without spills.
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
template <int KP>
__global__ __launch_bounds__(kTW, (KP <= 8 ? 2 : 1)) void k_packed_nm(const TrajDev* __restrict__ trajs,
                                                                      int64_t step0, int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.frame)
    packed_body<KP, true, 2>(T, 0, step0, nchunk);
  else
    packed_body<KP, false, 2>(T, 0, step0, nchunk);
}
template <int KP>
__global__ __launch_bounds__(kTW, (KP <= 8 ? 2 : 1)) void k_packed_nm_prologue(const TrajDev* __restrict__ trajs,
                                                                               int64_t step0, int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.frame)
    packed_body<KP, true, 2>(T, 1, step0, nchunk);
  else
    packed_body<KP, false, 2>(T, 1, step0, nchunk);
}

// Kinds 0 and 1 with the Gram terms on the matrix cores, arithmetic mode GM
// (0 FP64, 1 FP32, 2 BF16x3; the stencil, the jump assembly, the solve and
// the RK4 state stay FP64) and NS output tiles per wave.  Two tiles per wave
// (M <= 21) keep two workgroups per CU in registers; three (M <= 32) come
// with layer tiles that hold one workgroup per CU in LDS anyway.
template <int GM, int NS>
__device__ __forceinline__ void packed_mg_body(const TrajDev& T, int prologue, int64_t step0, int64_t nchunk) {
  if (prologue) {
    packed_body<2, false, 0, GM, NS>(T, 1, step0, nchunk);
  } else if (T.mkind == 1) {
    if (T.frame)
      packed_body<2, true, 1, GM, NS>(T, 0, step0, nchunk);
    else
      packed_body<2, false, 1, GM, NS>(T, 0, step0, nchunk);
  } else if (T.frame) {
    packed_body<2, true, 0, GM, NS>(T, 0, step0, nchunk);
  } else {
    packed_body<2, false, 0, GM, NS>(T, 0, step0, nchunk);
  }
}
template <int GM>
__global__ __launch_bounds__(kTW, 2) void k_packed_mg(const TrajDev* __restrict__ trajs, int64_t step0,
                                                      int64_t nchunk) {
  packed_mg_body<GM, 2>(trajs[blockIdx.x], 0, step0, nchunk);
}
template <int GM>
__global__ __launch_bounds__(kTW, 2) void k_packed_mg_prologue(const TrajDev* __restrict__ trajs, int64_t step0,
                                                               int64_t nchunk) {
  packed_mg_body<GM, 2>(trajs[blockIdx.x], 1, step0, nchunk);
}
template <int GM>
__global__ __launch_bounds__(kTW) void k_packed_mg3(const TrajDev* __restrict__ trajs, int64_t step0,
                                                    int64_t nchunk) {
  packed_mg_body<GM, 3>(trajs[blockIdx.x], 0, step0, nchunk);
}
template <int GM>
__global__ __launch_bounds__(kTW) void k_packed_mg3_prologue(const TrajDev* __restrict__ trajs, int64_t step0,
                                                             int64_t nchunk) {
  packed_mg_body<GM, 3>(trajs[blockIdx.x], 1, step0, nchunk);
}
template <int GM>
inline const void* packed_mg_kernel(int slots, bool prologue) {
  if (slots <= 2 || GM == 2)
    return prologue ? (const void*)k_packed_mg_prologue<GM> : (const void*)k_packed_mg<GM>;
  return prologue ? (const void*)k_packed_mg3_prologue<GM> : (const void*)k_packed_mg3<GM>;
}

constexpr int kPackedKP[] = {2, 3, 5, 8, 12, 16};
// The packed kernel for block size kp (vector-ALU Gram terms, gm < 0) or
// matrix-core mode gm; nm: the normal-mode model.
// slots: output tiles per wave of the matrix-core modes (mg_slots of the largest rank).
template <int I = 0>
inline const void* packed_kernel(int kp, bool prologue, bool nm = false, int gm = -1, int slots = 2) {
  if (gm == 0) return packed_mg_kernel<0>(slots, prologue);
  if (gm == 1) return packed_mg_kernel<1>(slots, prologue);
  if (gm == 2) return packed_mg_kernel<2>(slots, prologue);
  if constexpr (I + 1 < (int)(sizeof(kPackedKP) / sizeof(int))) {
    if (kp > kPackedKP[I]) return packed_kernel<I + 1>(kp, prologue, nm);
  }
  if (nm) return prologue ? (const void*)k_packed_nm_prologue<kPackedKP[I]> : (const void*)k_packed_nm<kPackedKP[I]>;
  return prologue ? (const void*)k_packed_prologue<kPackedKP[I]> : (const void*)k_packed<kPackedKP[I]>;
}

// Chunks of layer-split trajectories: blockIdx.x -> (trajectory, part) by the
// tile map.  Their prologue is the one-workgroup kernel (the Gram terms of
// the initial state are formed once per run).  One workgroup per CU suffices
// (few trajectories are split at a time), so the normal-mode kernel keeps its
// registers free of spills.
template <int KP>
__global__ __launch_bounds__(kTW) void k_packed_split(const TrajDev* __restrict__ trajs,
                                                      const int2* __restrict__ tilemap, int64_t step0,
                                                      int64_t nchunk) {
  const int2 tw = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tw.x];
  if (T.mkind == 1) {
    if (T.frame)
      packed_body<KP, true, 1, -1, 2, true>(T, 0, step0, nchunk, tw.y);
    else
      packed_body<KP, false, 1, -1, 2, true>(T, 0, step0, nchunk, tw.y);
  } else if (T.frame) {
    packed_body<KP, true, 0, -1, 2, true>(T, 0, step0, nchunk, tw.y);
  } else {
    packed_body<KP, false, 0, -1, 2, true>(T, 0, step0, nchunk, tw.y);
  }
}
template <int KP>
__global__ __launch_bounds__(kTW) void k_packed_split_nm(const TrajDev* __restrict__ trajs,
                                                         const int2* __restrict__ tilemap, int64_t step0,
                                                         int64_t nchunk) {
  const int2 tw = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tw.x];
  if (T.frame)
    packed_body<KP, true, 2, -1, 2, true>(T, 0, step0, nchunk, tw.y);
  else
    packed_body<KP, false, 2, -1, 2, true>(T, 0, step0, nchunk, tw.y);
}
template <int I = 0>
inline const void* packed_split_kernel(int kp, bool nm) {
  if constexpr (I + 1 < (int)(sizeof(kPackedKP) / sizeof(int))) {
    if (kp > kPackedKP[I]) return packed_split_kernel<I + 1>(kp, nm);
  }
  return nm ? (const void*)k_packed_split_nm<kPackedKP[I]> : (const void*)k_packed_split<kPackedKP[I]>;
}

// Zero the barrier flags (A, B and C) of the split trajectories trajs[0 .. n).
__global__ void k_reset_split(const TrajDev* __restrict__ trajs, int n) {
  if ((int)blockIdx.x >= n) return;
  const TrajDev& T = trajs[blockIdx.x];
  for (int i = threadIdx.x; i < T.P * kFlagStride; i += blockDim.x) {
    T.flagA[i] = 0u;
    T.flagB[i] = 0u;
    T.flagB[T.P * kFlagStride + i] = 0u;
  }
}

}  // namespace lrk
