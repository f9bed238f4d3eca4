// Persistent on-chip RK4 integrator (gfx950).
//
// A trajectory is split into P workgroups, each owning `rt` whole resonator
// layers (the jump operators never leave a layer).  The state of a workgroup's
// rows -- the base B_n and the RK4 accumulator in registers, the current stage
// input in LDS -- stays on chip for a whole chunk of steps.  Per RK4 stage:
//
//   1. solve G X_k = C_k for the reduced G = S^S, C_k = S^ L_k S of the stage
//      input (FP64 Gauss-Jordan elimination of the augmented [G | C_1 C_2],
//      held in the registers of two waves, a column per lane and half of the
//      rows per wave, the multipliers read across lanes, one barrier per
//      pivot); W_k = X_k^
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

#include <type_traits>

#include "lr_device.h"

namespace lrk {

constexpr int kPW = 512;  // threads per workgroup
constexpr int kDriveWin = 32;  // steps per refill of the drive table (4 stages each, one thread per stage)
// The kernel is instantiated for ROWS = 2 and 3 rows of one column per
// thread (ceil(rows / (kPW / M)) <= ROWS); 2 keeps every value in registers.
constexpr int kMaxRowsPerThread = 3;
constexpr size_t kPersistLdsMax = 159 * 1024;  // dynamic LDS (160 KB less the static part)

// Dynamic LDS bytes of k_persist for rt layers of L rows at rank M and P
// workgroups: stage input with halos, W, an area of 4 x 256 complex (with W,
// the LDS solver's augmented matrix), per-row jump coefficients, square-root
// table.
__host__ __device__ inline size_t persist_lds_bytes(int rt, int L, int M, int /* P */) {
  return (size_t)((rt + 2) * L * M + 2 * M * M + 4 * 256) * 16 + (size_t)(2 * rt * L + L + rt + 1) * 8;
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

// Arithmetic of the operator applications, the jump assembly and the
// Gram/cross partials by precision mode PREC (0 = FP64, 1 = FP32,
// 2 = BF16x3).  In FP32 the operands are rounded to FP32 and products and
// sums are FP32.  In BF16x3 each FP32 operand is split into BF16 parts
// x = x_h + x_m + ..., and a product is formed from its three leading part
// products x_h y_m + x_m y_h + x_h y_h (each exact in FP32) with FP32
// accumulation -- the split-BF16 product of matrix engines, evaluated here on
// the vector ALU.  The M x M solve, the cross-workgroup reduction of the
// partials and the RK4 state and accumulation stay FP64 in every mode.
// Reduced arithmetic needs the rank padding well above its rounding: with
// padding columns of norm 1e-6 (G's smallest eigenvalues 1e-12 of its
// largest) FP32 products drive the padded directions to O(1) errors, with the
// paper's padding weight 1e-5 they stay at the 1e-6 level.
// Arithmetic of the Gram G = B^B by mode: FP64 and FP32 as the mode; FP64
// for BF16x3, whose ~16-bit products do not resolve G's smallest eigenvalues
// (padding weight 1e-5 of the largest: a Schur complement turns
// non-positive), while the cross products C_k, the operator applications and
// the assembly take the split-BF16 arithmetic.
#define LR_GRAM_PREC(p) ((p) == 2 ? 0 : (p))
__device__ __forceinline__ float bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

template <int PREC>
struct Ar {  // FP64
  typedef double R;
  typedef double2 C;
  static __device__ __forceinline__ R in(double v) { return v; }
  static __device__ __forceinline__ C in(double2 v) { return v; }
  static __device__ __forceinline__ double2 out(C v) { return v; }
  static __device__ __forceinline__ R fma(R a, R b, R c) { return ::fma(a, b, c); }
  static __device__ __forceinline__ R shfl_xor(R v, int m) { return __shfl_xor(v, m); }
};
template <>
struct Ar<1> {  // FP32
  typedef float R;
  typedef float2 C;
  static __device__ __forceinline__ R in(double v) { return (float)v; }
  static __device__ __forceinline__ C in(double2 v) { return make_float2((float)v.x, (float)v.y); }
  static __device__ __forceinline__ double2 out(C v) { return make_double2(v.x, v.y); }
  static __device__ __forceinline__ R fma(R a, R b, R c) { return fmaf(a, b, c); }
  static __device__ __forceinline__ R shfl_xor(R v, int m) { return __shfl_xor(v, m); }
};
template <>
struct Ar<2> : Ar<1> {  // BF16x3
  static __device__ __forceinline__ R fma(R a, R b, R c) {
    const float ah = bf16_rne(a), am = bf16_rne(a - ah);
    const float bh = bf16_rne(b), bm = bf16_rne(b - bh);
    c = fmaf(am, bh, c);
    c = fmaf(ah, bm, c);
    return fmaf(ah, bh, c);
  }
};

// complex forms in the arithmetic of A
template <class A>
__device__ __forceinline__ typename A::C amac(typename A::C acc, typename A::C a, typename A::C b) {
  acc.x = A::fma(a.x, b.x, acc.x);
  acc.x = A::fma(-a.y, b.y, acc.x);
  acc.y = A::fma(a.x, b.y, acc.y);
  acc.y = A::fma(a.y, b.x, acc.y);
  return acc;
}
template <class A>
__device__ __forceinline__ typename A::C ajmac(typename A::C acc, typename A::C a, typename A::C b) {
  acc.x = A::fma(a.x, b.x, acc.x);
  acc.x = A::fma(a.y, b.y, acc.x);
  acc.y = A::fma(a.x, b.y, acc.y);
  acc.y = A::fma(-a.y, b.x, acc.y);
  return acc;
}
template <class A>
__device__ __forceinline__ typename A::C afma(typename A::R s, typename A::C a, typename A::C acc) {
  acc.x = A::fma(s, a.x, acc.x);
  acc.y = A::fma(s, a.y, acc.y);
  return acc;
}
template <class A>
__device__ __forceinline__ typename A::C azero() {
  typename A::C z;
  z.x = 0;
  z.y = 0;
  return z;
}

__device__ __forceinline__ void flag_arrive(g_u32* flag, uint32_t value) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until flags[w * kFlagStride] >= target for all w < P.  Returns false
// if the wait expired or the group was aborted.
__device__ __forceinline__ bool flag_wait(const TrajDev& T, const g_u32* flags, uint32_t target, int* s_ok) {
  g_u32* abort_flag = (g_u32*)T.abort_flag;
  const uint32_t limit = T.spin_limit ? T.spin_limit : kSpinLimit;
  target += T.wait_bias;
  if (threadIdx.x < 64) {
    bool ok = true;
    for (int w = threadIdx.x; w < T.P && ok; w += 64) {
      uint32_t n = 0;
      while (__hip_atomic_load(flags + (size_t)w * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             target) {
        // the abort flag is read on every 16th poll only, so that a poll is one
        // memory round trip
        if (++n > limit ||
            ((n & 15u) == 0u && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
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

// v + (v of lane l ^ 32): the two halves of a wave; both lanes get the same
// bits (the sum is commutative)
template <class A>
__device__ __forceinline__ typename A::C add_wave_halves(typename A::C v) {
  v.x += A::shfl_xor(v.x, 32);
  v.y += A::shfl_xor(v.y, 32);
  return v;
}

// Gram / cross partials of the tile (rows x M in LDS) -> dst[3 M^2]:
//   G[i][j]   = sum_rho conj(O[rho][i]) O[rho][j]
//   C_1[i][j] = sum_rho conj(O[rho][i]) sqrt(kappa (f+1)) O[rho+1][j]      (f+1 < d_f)
//   C_2[i][j] = sum_rho conj(O[rho][i]) sqrt(gamma (q+1)) O[rho+d_f][j]    (q+1 < d_q)
// c1row / c2row hold those coefficients per row and 0 where the jump leaves
// the mode (the row read there is a finite neighbour in the tile or halo).
// Lanes l and l + 32 of a wave own the entries (i0, j), (i0 + 1, j) of all
// three matrices; each sums one half of the rows (in order) and the halves
// are added across the wave.  Consecutive lanes of a half take consecutive
// j, so the row reads of a half are bank-conflict free.  Every lane of the
// block takes the same number of passes, so both partners are always present.
template <int PREC, int GP>
__device__ __forceinline__ void persist_partials(const TrajDev& T, const double2* tile, int R, const double* c1row,
                                                 const double* c2row, g_double2* dst) {
  typedef Ar<PREC> A;
  typedef typename A::C C;
  typedef Ar<GP> G;  // arithmetic of the Gram G
  const int M = T.M, MM = M * M, d_f = T.d_f;
  const int nu = ((M + 1) >> 1) * M;   // (i pair, j) units
  const int Rh = (R + 1) >> 1;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  for (int u0 = 0; u0 < nu; u0 += kPW / 2) {
    const int uu = u0 + (int)(threadIdx.x >> 6) * 32 + (lane & 31);
    const bool valid = uu < nu;
    const int u = valid ? uu : 0;
    const int ip = u / M, j = u - ip * M;
    const int i0 = 2 * ip, i1 = min(i0 + 1, M - 1);
    const int ra = h ? Rh : 0, rb = h ? R : Rh;
    typename G::C g0 = azero<G>(), g1 = g0;
    C a0 = azero<A>(), a1 = a0, b0 = a0, b1 = a0;
    for (int r = ra; r < rb; ++r) {
      const double2* row = tile + r * M;
      const double2 xd0 = row[i0], xd1 = row[i1], yd = row[j];
      g0 = ajmac<G>(g0, G::in(xd0), G::in(yd));
      g1 = ajmac<G>(g1, G::in(xd1), G::in(yd));
      const C x0 = A::in(xd0), x1 = A::in(xd1);
      const C yf = A::in(cscale(c1row[r], row[M + j]));
      const C yq = A::in(cscale(c2row[r], row[d_f * M + j]));
      a0 = ajmac<A>(a0, x0, yf);
      a1 = ajmac<A>(a1, x1, yf);
      b0 = ajmac<A>(b0, x0, yq);
      b1 = ajmac<A>(b1, x1, yq);
    }
    g0 = add_wave_halves<G>(g0);
    g1 = add_wave_halves<G>(g1);
    a0 = add_wave_halves<A>(a0);
    a1 = add_wave_halves<A>(a1);
    b0 = add_wave_halves<A>(b0);
    b1 = add_wave_halves<A>(b1);
    if (valid && h == 0) {
      const int o0 = i0 * M + j;
      st_ag(dst + o0, G::out(g0));
      st_ag(dst + MM + o0, A::out(a0));
      st_ag(dst + 2 * MM + o0, A::out(b0));
      if (i0 + 1 < M) {
        st_ag(dst + o0 + M, G::out(g1));
        st_ag(dst + MM + o0 + M, A::out(a1));
        st_ag(dst + 2 * MM + o0 + M, A::out(b1));
      }
    }
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

// W_k = X_k^ with X_k = G^-1 C_k (G Hermitian positive definite): Gauss-Jordan
// elimination of the augmented M x 3M matrix [G | C_1 | C_2] without
// pivoting, down to [I | X_1 | X_2].  Pivot k takes every row i != k to
// row_i - A[i][k] row_k / p and row k to row_k / p, p = Re A[k][k]: these are
// the pivots of G = L D L^ (all positive iff G is positive definite, so a
// non-positive one is reported like a failed Cholesky), the imaginary part of
// the diagonal entry being rounding (G is Hermitian).  The right-hand sides
// are eliminated directly: no inverse of G is formed (an explicit inverse
// followed by a product carries cond(G) times more rounding into X_k, and G
// is ill-conditioned through the rank padding).
//
// The elimination runs in two waves: lane c of wave w (w = 0, 1) holds rows
// kWsHalf w .. kWsHalf w + kWsHalf - 1 of column c of the augmented
// [G | C_1 | C_2] (3M <= 64 columns) in registers.  At pivot k the
// multipliers A[i][k] of a wave's rows are the registers of its lane k, read
// as wave-uniform values (v_readlane); the pivot row A[k][c] comes from the
// wave that holds row k, which writes it to LDS right after updating it in the
// previous pivot; one workgroup barrier per pivot, taken by every wave at the
// same points (the other waves only pass the barriers).
constexpr int kWsHalf = 10;           // rows per solver wave
constexpr int kWsRows = 2 * kWsHalf;  // ranks M <= 20
constexpr int kSolveWaves = 4;
constexpr int kWsLds = 4 * 64;  // LDS (complex entries): the pivot-row buffers of the register solver; the LDS
                                // solver's augmented matrix reaches into this area (3 M^2 <= 2 M^2 + 1024 at M = 32)
__host__ __device__ inline bool ws_fits(int M) { return M <= kWsRows && 3 * M <= 64; }

struct WsRegs {
  double2 a[kWsHalf];
};

// Loads of the lane's rows of its column of the reduced [G | C_1 | C_2] (each
// M x M row-major; issued early so that their latency overlaps other work).
// Every thread calls it; threads outside the two solver waves load nothing.
__device__ __forceinline__ void wsolve_load(const g_double2* red, int M, WsRegs& R) {
  const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const bool act = wv < 2 && lane < 3 * M;
  const int blk = act ? lane / M : 0, col = act ? lane - blk * M : 0;
  const g_double2* src = red + (size_t)blk * M * M + col;
#pragma unroll
  for (int r = 0; r < kWsHalf; ++r) {
    const int row = wv * kWsHalf + r;
    R.a[r] = make_double2(0.0, 0.0);
    if (act && row < M) R.a[r] = ld_ag(src + (size_t)row * M);
  }
}

// Value of v in lane `lane` of the wave (a uniform result).
__device__ __forceinline__ double ws_readlane(double v, int lane) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane), hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Row update of pivot k in a lane's column: v <- v - A[i][k] pc, the
// multiplier A[i][k] being the same row's register in lane k.
__device__ __forceinline__ void ws_update(double2& v, int k, double2 pc) {
  const double mx = ws_readlane(v.x, k), my = ws_readlane(v.y, k);
  v.x = fma(-mx, pc.x, v.x);
  v.x = fma(my, pc.y, v.x);
  v.y = fma(-mx, pc.y, v.y);
  v.y = fma(-my, pc.x, v.y);
}

// Elimination (every thread of the workgroup calls it; it passes M workgroup
// barriers in every thread).  prow: 2 x 64 complex entries of LDS.  Writes
// W_k[i][j] = conj(X_k[j][i]) to Wl (W_1 then W_2, M x M row-major each).
// s_nonfinite (LDS, zero on entry) is set on a non-finite input and then
// nothing is eliminated; *s_bad receives the first non-positive pivot or -1.
// The caller synchronises the workgroup before reading Wl or the flags.  Rows
// past M are zero and stay zero; pivot k and the register rows are
// compile-time constants of the unrolled loops.
__device__ __forceinline__ void wsolve_run(WsRegs& R, double2* prow, double2* Wl, int M, int* s_nonfinite,
                                           int* s_bad) {
  const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const bool solver = wv < 2;  // uniform per wave
  bool bad = false;
  if (solver) {
#pragma unroll
    for (int r = 0; r < kWsHalf; ++r) bad = bad || !isfinite(R.a[r].x) || !isfinite(R.a[r].y);
  }
  if (bad) *s_nonfinite = 1;
  if (threadIdx.x == 0) *s_bad = -1;
  if (wv == 0) prow[lane] = R.a[0];  // row 0 of the pivot-row buffer 0
  __syncthreads();
  if (*s_nonfinite) return;  // uniform over the workgroup
  // every pivot runs; the first non-positive one is recorded and the caller discards the result
  int first_bad = -1;
#pragma unroll
  for (int k = 0; k < kWsRows; ++k) {
    if (k < M) {  // uniform
      if (k > 0) __syncthreads();  // row k in buffer k & 1
      if (solver) {
        const double2 pr = prow[(k & 1) * 64 + lane];  // A[k][c]
        const double piv = ws_readlane(pr.x, k);        // A[k][k]: lane k
        if (!(piv > 0.0) && first_bad < 0) first_bad = k;
        const double rinv = pivot_rcp(piv > 0.0 ? piv : 1.0);
        const double2 pc = make_double2(pr.x * rinv, pr.y * rinv);  // row k of the result, this column
        auto body = [&](auto rbc) {
          constexpr int RB = decltype(rbc)::value;  // first row of the wave
          // row k + 1 first when the wave holds it: it goes to the other buffer for the next pivot
          if (k + 1 >= RB && k + 1 < RB + kWsHalf) {  // compile time
            ws_update(R.a[k + 1 - RB], k, pc);
            prow[((k + 1) & 1) * 64 + lane] = R.a[k + 1 - RB];
          }
#pragma unroll
          for (int r = 0; r < kWsHalf; ++r) {  // compile time; rows past M are zero and stay zero
            if (RB + r == k) R.a[r] = pc;
            else if (RB + r != k + 1) ws_update(R.a[r], k, pc);
          }
        };
        if (wv == 0) body(std::integral_constant<int, 0>{});
        else body(std::integral_constant<int, kWsHalf>{});
      }
    }
  }
  if (threadIdx.x == 0) *s_bad = first_bad;
  // right-hand-side lanes hold X_k[:, i]: W_k[i][j] = conj(X_k[j][i])
  if (solver && first_bad < 0 && lane >= M && lane < 3 * M) {
    const int cc = lane - M, kk = cc < M ? 0 : 1, i = cc - kk * M;
    double2* dst = Wl + (size_t)kk * M * M + (size_t)i * M;
#pragma unroll
    for (int r = 0; r < kWsHalf; ++r) {
      const int row = wv * kWsHalf + r;
      if (row < M) dst[row] = make_double2(R.a[r].x, -R.a[r].y);
    }
  }
}

// The same elimination for ranks whose columns do not fit a solver wave's
// registers (M >= 21 with 10 register rows per lane): the M x 3M matrix sits in
// LDS and the whole workgroup takes each pivot, one barrier per pivot.  The
// pivot rows are left unscaled -- pivot k takes row i != k to
// row_i - (A[i][k] / p) row_k, which reads row k and column k but writes
// neither -- so that a pivot needs no second barrier; the result rows are
// divided by their pivots at the end (X_k = D^-1 [eliminated C_k], D the
// pivots).  Aug: 3 M^2 complex entries of LDS.  Returns like wsolve_run
// through the same flags (every thread calls it; the flags are valid after
// the caller's barrier).
__device__ __forceinline__ void lsolve_run(const g_double2* red, double2* Aug, double2* Wl, int M,
                                           int* s_nonfinite, int* s_bad) {
  const int MM = M * M, C3 = 3 * M, tot = M * C3, tid = threadIdx.x;
  bool bad = false;
  for (int e = tid; e < tot; e += kPW) {  // Aug[i][c] = [G | C_1 | C_2][i][c]
    const int i = e / C3, c = e - i * C3, blk = c / M;
    const double2 v = ld_ag(red + (size_t)blk * MM + i * M + (c - blk * M));
    bad = bad || !isfinite(v.x) || !isfinite(v.y);
    Aug[e] = v;
  }
  if (bad) *s_nonfinite = 1;
  if (tid == 0) *s_bad = -1;
  __syncthreads();
  if (*s_nonfinite) return;
  for (int k = 0; k < M; ++k) {
    const double piv = Aug[k * C3 + k].x;
    if (!(piv > 0.0)) {  // uniform
      if (tid == 0) *s_bad = k;
      return;
    }
    const double rp = pivot_rcp(piv);
    for (int e = tid; e < tot; e += kPW) {
      const int i = e / C3, c = e - i * C3;
      if (c > k && i != k) {
        const double2 a = Aug[i * C3 + k], b = Aug[k * C3 + c];
        const double2 l = make_double2(a.x * rp, a.y * rp);
        double2 v = Aug[e];
        v.x = fma(-l.x, b.x, v.x);
        v.x = fma(l.y, b.y, v.x);
        v.y = fma(-l.x, b.y, v.y);
        v.y = fma(-l.y, b.x, v.y);
        Aug[e] = v;
      }
    }
    __syncthreads();
  }
  // X_k[j][i] = Aug[j][M (k + 1) + i] / p_j;  W_k[i][j] = conj(X_k[j][i]) (Wl aliases Aug: read, then write)
  constexpr int kWPer = (2 * kMaxM * kMaxM + kPW - 1) / kPW;
  double2 w[kWPer];
#pragma unroll
  for (int u = 0; u < kWPer; ++u) {
    const int e = tid + u * kPW;
    if (e < 2 * MM) {
      const int kk = e / MM, o = e - kk * MM, i = o / M, j = o - i * M;
      const double r = pivot_rcp(Aug[j * C3 + j].x);
      const double2 x = Aug[j * C3 + M * (kk + 1) + i];
      w[u] = make_double2(x.x * r, -x.y * r);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kWPer; ++u) {
    const int e = tid + u * kPW;
    if (e < 2 * MM) Wl[e] = w[u];
  }
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

// The kernel body: the prologue (partials and reduction of the initial stage
// input, no step) or a chunk of nchunk RK4 steps from step0.
template <int ROWS, int GE, int PREC>
__device__ __forceinline__ void persist_body(const TrajDev* __restrict__ trajs, const int2* __restrict__ tilemap,
                                             int prologue, int64_t step0, int64_t nchunk) {
  extern __shared__ double2 lds[];
  __shared__ int s_ok;
  __shared__ int s_nonfinite;
  __shared__ int s_bad;
  __shared__ double s_part[kPW / 64];
  // per stage of kDriveWin steps: d(t) and, in the drive frame, e^{i w_d t}, e^{2 i w_d t}
  __shared__ double s_dtab[4 * kDriveWin][5];

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
  double2* WS = Wl + 2 * MM;                      // kSolveWaves x kWsLds: the LDS solver's matrix runs on into it
  double* c1row = reinterpret_cast<double*>(WS + kSolveWaves * kWsLds);
  double* c2row = c1row + rt * L;
  double* sqt = c2row + rt * L;                   // sqrt(n), n < nq; then sqrt(r0 + k), k <= rt
  const int nq = max(d_q, d_f);
  const double* sqr = sqt + nq;

  // halo layers start at zero: the jump partials read one neighbour row past
  // the tile edge with a zero coefficient
  for (int idx = tid; idx < 2 * LM; idx += kPW) SL[idx < LM ? idx : (size_t)(R + L) * M + (idx - LM)] = make_double2(0.0, 0.0);
  for (int rl = tid; rl < R; rl += kPW) {
    const int rem = rl % L, q = rem / d_f, f = rem - q * d_f;
    c1row[rl] = f + 1 < d_f ? sqrt(T.kappa * (double)(f + 1)) : 0.0;
    c2row[rl] = q + 1 < d_q ? sqrt(T.gamma * (double)(q + 1)) : 0.0;
  }
  for (int n = tid; n < nq + rt + 1; n += kPW) sqt[n] = sqrt((double)(n < nq ? n : r0 + (n - nq)));

  // element mapping: column j, rows rg, rg + NG, ...
  const int NG = kPW / M;
  const int j = tid % M, rg = tid / M;
  const bool active = rg < NG;

  double2 base[ROWS], acc[ROWS], o_new[ROWS];
  int rq[ROWS], rf[ROWS], rr[ROWS];  // mode indices (q, f, r - r0) of the thread's rows
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int rl = rg + k * NG;
    const int lr = rl / L, rem = rl - lr * L;
    rq[k] = rem / d_f;
    rf[k] = rem - rq[k] * d_f;
    rr[k] = lr;
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

  // Exchange after group barrier A for the stage input of parity `par`: the
  // two halo layers (published boundary layers of the neighbours; zero past
  // the ends) into SL, and the slice reduction of the partials.  Each slice
  // entry is summed by a 16-lane group straight from global memory: lane l
  // adds workgroups l, l + 16, ... in order, then a butterfly over the group,
  // so the order depends on P only.  The halo loads and the first batch of
  // partial loads are in flight together.
  auto exchange = [&](int par, bool halo) {
    const g_double2* hsrc = SPg + (size_t)par * NMn;
    const size_t lo_base = r0 > 0 ? (size_t)(row0 - L) * M : 0;
    const size_t hi_base = r1 < d_r ? (size_t)(row0 + R) * M : 0;
    const g_double2* psrc = PARTg + (size_t)par * P * npe + e0;
    g_double2* dst = REDg + (size_t)par * npe + e0;
    const int nh = halo ? 2 * LM : 0;
    const int sub = tid & 15, grp = tid >> 4;
    constexpr int kPB = 8;  // partial loads per lane in flight
    for (int b = 0; b * 4 * kPW < nh || b * (kPW / 16) < ne; ++b) {
      const int hb = b * 4 * kPW, e = b * (kPW / 16) + grp;
      const bool doh = hb < nh, dop = b * (kPW / 16) < ne;  // uniform
      const int ec = min(e, ne - 1);
      double2 hv[4], pv[kPB];
      if (doh) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = min(hb + tid + u * kPW, nh - 1);
          const bool lo = idx < LM;
          hv[u] = ld_ag(hsrc + (lo ? lo_base : hi_base) + (lo ? idx : idx - LM));
        }
      }
      double2 sum = make_double2(0.0, 0.0);
      for (int pb = 0; dop && pb < P; pb += 16 * kPB) {
#pragma unroll
        for (int u = 0; u < kPB; ++u) pv[u] = ld_ag(psrc + (size_t)min(pb + sub + 16 * u, P - 1) * npe + ec);
        if (doh && pb == 0) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int idx = hb + tid + u * kPW;
            if (idx < nh) {
              const bool lo = idx < LM;
              const int off = lo ? idx : idx - LM;
              const bool have = lo ? r0 > 0 : r1 < d_r;
              const double2 val = have ? hv[u] : make_double2(0.0, 0.0);
              if (lo) SL[off] = val;
              else SL[(size_t)(R + L) * M + off] = val;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kPB; ++u)
          if (pb + sub + 16 * u < P) sum = cadd(sum, pv[u]);
      }
      if (doh && !dop) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = hb + tid + u * kPW;
          if (idx < nh) {
            const bool lo = idx < LM;
            const int off = lo ? idx : idx - LM;
            const bool have = lo ? r0 > 0 : r1 < d_r;
            const double2 val = have ? hv[u] : make_double2(0.0, 0.0);
            if (lo) SL[off] = val;
            else SL[(size_t)(R + L) * M + off] = val;
          }
        }
      }
      if (dop) {
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
          sum.x += __shfl_xor(sum.x, off, 16);
          sum.y += __shfl_xor(sum.y, off, 16);
        }
        if (sub == 0 && e < ne) st_ag(dst + e, sum);
      }
    }
  };

  if (prologue) {
    const int64_t g = 4 * step0;
    const int p = (int)(g & 1);
    __syncthreads();
    persist_partials<PREC, LR_GRAM_PREC(PREC)>(T, tile, R, c1row, c2row, PARTg + ((size_t)p * P + w) * npe);
    publish_boundary(tile, SPg + (size_t)p * NMn, row0, R, L, M);
    flag_arrive(myA, (uint32_t)(g + 1));
    bool ok = flag_wait(T, flagA, (uint32_t)(g + 1), &s_ok);
    if (ok) {
      exchange(p, false);
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
  {  // halo layers of the first stage input (published by the prologue or the previous chunk)
    const int par = (int)((4 * step0) & 1);
    const g_double2* hsrc = SPg + (size_t)par * NMn;
    const size_t lo_base = r0 > 0 ? (size_t)(row0 - L) * M : 0;
    const size_t hi_base = r1 < d_r ? (size_t)(row0 + R) * M : 0;
    for (int idx = tid; idx < 2 * LM; idx += kPW) {
      const bool lo = idx < LM;
      const int off = lo ? idx : idx - LM;
      const bool have = lo ? r0 > 0 : r1 < d_r;
      const double2 val = have ? ld_ag(hsrc + (lo ? lo_base : hi_base) + off) : make_double2(0.0, 0.0);
      if (lo) SL[off] = val;
      else SL[(size_t)(R + L) * M + off] = val;
    }
  }
  const double dt = T.dt;
  // time of stage s of step n: t_n + c_s dt with c = 0, 1/2, 1/2, 1 and
  // t_n = t0 + (step_base + n) dt
  auto stage_time = [&](int64_t step, int s) {
    const double c = (s == 0) ? 0.0 : (s == 3 ? 1.0 : 0.5);
    return T.t0 + (double)(T.step_base + step) * dt + c * dt;
  };
  // drive values of the stages of the next kDriveWin steps from step, one
  // stage time per thread (any pulse kind costs the same per stage)
  auto fill_drive = [&](int64_t step) {
    __syncthreads();
    if (tid < 4 * kDriveWin) {
      const double t = stage_time(step + tid / 4, tid % 4);
      s_dtab[tid][0] = drive_at(T, t);
      if (T.frame) {
        const double2 e1 = frame_phase(T.w_d, t), e2 = frame_phase(2.0 * T.w_d, t);
        s_dtab[tid][1] = e1.x;
        s_dtab[tid][2] = e1.y;
        s_dtab[tid][3] = e2.x;
        s_dtab[tid][4] = e2.y;
      }
    }
  };
  const int64_t nrun = max((int64_t)0, min(nchunk, T.nsteps - step0));  // trajectories of a batch end apart
  bool ok = true;
  bool failed = false;
  int64_t n = 0;
  for (; n < nrun && ok && !failed; ++n) {
    const int64_t step = step0 + n;
    if (n % kDriveWin == 0) fill_drive(step);
    for (int s = 0; s < 4; ++s) {
      const int64_t g = 4 * step + s;
      const int p = (int)(g & 1);
      const int ds = (int)(n % kDriveWin) * 4 + s;
      if (tid == 0) s_nonfinite = 0;
      __syncthreads();  // stage input tile and halo, drive table in LDS
      const double drv = s_dtab[ds][0];

      // (1) loads of the reduced G, C_k (solver waves of the register solver) in flight while
      // Z = H_eff(t) S is formed (with three register rows they are issued after it: registers)
      constexpr bool kWaveSolve = GE == 1, kEarlyLoad = kWaveSolve && ROWS == 2;
      WsRegs SR;
      if constexpr (kEarlyLoad) wsolve_load(REDg + (size_t)p * npe, M, SR);
      double2 z[ROWS];
      // Z rows of the thread, in the lab frame or the drive frame (one code
      // path per frame, chosen once per stage).  In the drive frame a
      // coupling or drive tap to a neighbour with dn more excitations carries
      // e^{-i w_d t dn}: the raising pairs (dn = -2) e^{2 i w_d t}, the
      // lowering pairs its conjugate, the drive taps d(t) e^{-+ i w_d t}, the
      // mixed pairs nothing.
      auto stencil = [&](auto rotc) {
        constexpr bool kRot = decltype(rotc)::value;
        double2 e1 = make_double2(1.0, 0.0), e2 = e1;
        if constexpr (kRot) {
          e1 = make_double2(s_dtab[ds][1], s_dtab[ds][2]);
          e2 = make_double2(s_dtab[ds][3], s_dtab[ds][4]);
        }
        const double2 e1c = make_double2(e1.x, -e1.y), e2c = make_double2(e2.x, -e2.y);
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
          const int rl = rg + k * NG;
          z[k] = make_double2(0.0, 0.0);
          if (active && rl < R) {
            // opaque per stage: values derived from the row indices are formed
            // here rather than held in registers across the whole chunk
            int q = rq[k], f = rf[k], rk = rr[k];
            asm volatile("" : "+v"(q), "+v"(f), "+v"(rk));
            const int r = r0 + rk;
            const double2* col = tile + j;  // row offsets relative to the tile (halo at -L, +R)
            const double2 b = col[rl * M];
            const double hr = T.w_q * q + 0.5 * T.alpha * q * (q - 1) + T.w_r * r + T.w_f * f;
            const double hi = -0.5 * (T.kappa * f + T.gamma * q);
            // sqrt(max(n, n +- 1)) of each mode: sqrt(n) downwards, sqrt(n + 1) upwards
            const double sq0 = sqt[q], sq1 = sqt[min(q + 1, nq - 1)];
            const double sf0 = sqt[f], sf1 = sqt[min(f + 1, nq - 1)];
            const double sr0 = sqr[rk], sr1 = sqr[rk + 1];
            const bool rlo = r > 0, rhi = r + 1 < d_r;
            typedef Ar<PREC> A;
            typedef typename A::R Rr;
            typename A::C zz = amac<A>(azero<A>(), A::in(make_double2(hr, hi)), A::in(b));
            auto tap = [&](double c, double2 ph, double2 nb) {  // real c in the lab frame
              if constexpr (kRot) zz = amac<A>(zz, A::in(cscale(c, ph)), A::in(nb));
              else zz = afma<A>((Rr)A::in(c), A::in(nb), zz);
            };
            auto tap0 = [&](double c, double2 nb) { zz = afma<A>((Rr)A::in(c), A::in(nb), zz); };
            if (q > 0) {
              if (rlo) tap(T.g * sq0 * sr0, e2, col[(rl - d_f - L) * M]);
              if (rhi) tap0(T.g * sq0 * sr1, col[(rl - d_f + L) * M]);
            }
            if (q + 1 < d_q) {
              if (rlo) tap0(T.g * sq1 * sr0, col[(rl + d_f - L) * M]);
              if (rhi) tap(T.g * sq1 * sr1, e2c, col[(rl + d_f + L) * M]);
            }
            if (f > 0) {
              if (rlo) tap(T.G * sf0 * sr0, e2, col[(rl - L - 1) * M]);
              if (rhi) tap0(T.G * sf0 * sr1, col[(rl + L - 1) * M]);
              tap(drv * sf0, e1, col[(rl - 1) * M]);
            }
            if (f + 1 < d_f) {
              if (rlo) tap0(T.G * sf1 * sr0, col[(rl - L + 1) * M]);
              if (rhi) tap(T.G * sf1 * sr1, e2c, col[(rl + L + 1) * M]);
              tap(drv * sf1, e1c, col[(rl + 1) * M]);
            }
            z[k] = A::out(zz);
          }
        }
      };
      if (T.frame) stencil(std::true_type{});
      else stencil(std::false_type{});
      // (2) W_k of this stage input (register solver: two solver waves, the others pass the
      // same barriers; LDS solver: the whole workgroup)
      {
        if constexpr (kWaveSolve) {
          if constexpr (!kEarlyLoad) wsolve_load(REDg + (size_t)p * npe, M, SR);
          wsolve_run(SR, WS, Wl, M, &s_nonfinite, &s_bad);
        } else {
          lsolve_run(REDg + (size_t)p * npe, Wl, Wl, M, &s_nonfinite, &s_bad);
        }
        __syncthreads();
        const int bad = s_nonfinite ? -2 : s_bad;
        if (bad != -1) {
          if (tid == 0) report(T, bad == -2 ? -5 /* LR_ERR_NONFINITE */ : -4 /* LR_ERR_GRAM_NOT_PD */, step);
          failed = true;
          break;
        }
      }

      // (3) k = -i Z + 1/2 sum_k (L_k S) W_k ; RK4 stage update.  The jump
      // term of a row is c1 (S W_1)[rho+1, j] + c2 (S W_2)[rho+d_f, j] (the
      // coefficient is 0 where the jump leaves the mode); the W entries of
      // column j are loaded once for all rows of the thread.
      {
        typedef Ar<PREC> A;
        typedef typename A::C C;
        const double2* y1[ROWS];
        const double2* y2[ROWS];
        C s1[ROWS], s2[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
          const int rl = min(rg + k * NG, R - 1);  // rows past the tile read a valid row, unused
          y1[k] = tile + (rl + 1) * M;
          y2[k] = tile + (rl + d_f) * M;
          s1[k] = azero<A>();
          s2[k] = s1[k];
        }
        const double2* W1 = Wl + j;
        const double2* W2 = Wl + MM + j;
        int i = 0;
        if (ROWS == 2)
          for (; i + 2 <= M; i += 2) {
            const C w1a = A::in(W1[i * M]), w1b = A::in(W1[(i + 1) * M]), w2a = A::in(W2[i * M]),
                    w2b = A::in(W2[(i + 1) * M]);
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
              s1[k] = amac<A>(amac<A>(s1[k], A::in(y1[k][i]), w1a), A::in(y1[k][i + 1]), w1b);
              s2[k] = amac<A>(amac<A>(s2[k], A::in(y2[k][i]), w2a), A::in(y2[k][i + 1]), w2b);
            }
          }
        for (; i < M; ++i) {
          const C w1a = A::in(W1[i * M]), w2a = A::in(W2[i * M]);
#pragma unroll
          for (int k = 0; k < ROWS; ++k) {
            s1[k] = amac<A>(s1[k], A::in(y1[k][i]), w1a);
            s2[k] = amac<A>(s2[k], A::in(y2[k][i]), w2a);
          }
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
          const int rl = rg + k * NG;
          if (active && rl < R) {
            const double2 zz = z[k];
            const double2 a = cfma(c2row[rl], A::out(s2[k]), cscale(c1row[rl], A::out(s1[k])));
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
      publish_boundary(tile, SPg + (size_t)pn * NMn, row0, R, L, M);  // stores drain during the partials
      persist_partials<PREC, LR_GRAM_PREC(PREC)>(T, tile, R, c1row, c2row, PARTg + ((size_t)pn * P + w) * npe);

      // (5) group barriers around the slice reduction
      flag_arrive(myA, (uint32_t)(g + 2));
      ok = flag_wait(T, flagA, (uint32_t)(g + 2), &s_ok);
      if (!ok) break;
      exchange(pn, true);
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

// Chunk of RK4 steps (the integrator proper) and prologue, as separate
// kernels so that timing tools see the step kernel alone.
// GE selects the solver: in the registers of two solver waves (1) or in LDS (2).
template <int ROWS, int GE, int PREC>
__global__ __launch_bounds__(kPW) void k_persist(const TrajDev* __restrict__ trajs,
                                                 const int2* __restrict__ tilemap, int64_t step0, int64_t nchunk) {
  persist_body<ROWS, GE, PREC>(trajs, tilemap, 0, step0, nchunk);
}
template <int ROWS, int GE, int PREC>
__global__ __launch_bounds__(kPW) void k_persist_prologue(const TrajDev* __restrict__ trajs,
                                                          const int2* __restrict__ tilemap, int64_t step0,
                                                          int64_t /* nchunk: same signature as k_persist */) {
  persist_body<ROWS, GE, PREC>(trajs, tilemap, 1, step0, 0);
}

// Kernel variant for ROWS rows per thread, rank M and precision mode: the
// register solver (GE = 1) when the lanes of a solver wave's columns fit the
// wave, else the LDS solver (GE = 2).
inline int persist_ge(int M) { return ws_fits(M) ? 1 : 2; }
template <int PREC>
inline const void* persist_kernel_p(int rows, int ge, bool prologue) {
  if (prologue) {
    if (rows <= 2)
      return ge <= 1 ? (const void*)k_persist_prologue<2, 1, PREC> : (const void*)k_persist_prologue<2, 2, PREC>;
    return ge <= 1 ? (const void*)k_persist_prologue<3, 1, PREC> : (const void*)k_persist_prologue<3, 2, PREC>;
  }
  if (rows <= 2) return ge <= 1 ? (const void*)k_persist<2, 1, PREC> : (const void*)k_persist<2, 2, PREC>;
  return ge <= 1 ? (const void*)k_persist<3, 1, PREC> : (const void*)k_persist<3, 2, PREC>;
}
inline const void* persist_kernel(int rows, int ge, bool prologue, int prec) {
  if (prec == 1) return persist_kernel_p<1>(rows, ge, prologue);
  if (prec == 2) return persist_kernel_p<2>(rows, ge, prologue);
  return persist_kernel_p<0>(rows, ge, prologue);
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
