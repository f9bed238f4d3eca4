// Adaptive-step integration of packed trajectories: the Dormand-Prince 5(4)
// pair with a per-trajectory step size.
//
// The paper integrates eq. "nosse" with an adaptive-timestep solver (main
// text, "Computational performance").  Here every trajectory of a batch runs
// in one workgroup, as in the packed schedule (lr_packed.hip), and carries its
// own time t and step proposal h across launches; a launch advances it to its
// next record time at or after the launch's end (t0 + (step0 + n) dt, records
// every obs_stride grid steps; with no records, the end of the integration),
// so that its steps land on its own record times only.  A trajectory may also
// be split over several workgroups (layer ranges, lr_packed.hip).  One step from (t, y) with k_1 = f(t, y):
//   Y_2 = y + hc a_21 k_1                      (a light pass, no stencil)
//   pass s = 2..6: k_s = f(t + c_s hc, Y_s),  Y_{s+1} = y + hc sum_j a_{s+1,j} k_j
//   pass 7:        k_7 = f(t + hc, Y_7)  with Y_7 the fifth-order solution,
//                  err = sqrt(mean_i |e_i|^2 / sc_i^2),  e = hc sum_j (b_j - bhat_j) k_j,
//                  sc_i = atol + rtol max(|y_i|, |Y_7,i|)   (one workgroup reduction)
// hc = min(h, t_end - t).  err <= 1 accepts (y <- Y_7, k_1 <- k_7: first same
// as last) and proposes h <- hc min(5, max(0.2, 0.9 err^(-1/5))) unless hc was
// shortened to hit t_end; a rejection shrinks h the same way, never grows it.
// Every pass forms the Gram terms and W_k of the next stage input as the RK4
// packed kernel does.  Each stage input lives in global memory (two
// alternating buffers), the k_j in seven buffers.
#include <hip/hip_runtime.h>

#include "lr_device.h"

namespace lrk {

struct AdaptDev {
  double rtol, atol;
  double2* K;      // [7][N*M] stage derivatives
  double* st;      // t, h
  int64_t* cnt;    // accepted, rejected, slot of k_1 (0 or 6), k_1 valid
};

// Dormand-Prince 5(4): nodes, stage rows (a_{s,j}, j < s), fifth-order weights
// (= the last row) and b - bhat
__constant__ double kDpC[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
__constant__ double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
__constant__ double kDpE[7] = {35.0 / 384.0 - 5179.0 / 57600.0,
                               0.0,
                               500.0 / 1113.0 - 7571.0 / 16695.0,
                               125.0 / 192.0 - 393.0 / 640.0,
                               -2187.0 / 6784.0 + 92097.0 / 339200.0,
                               11.0 / 84.0 - 187.0 / 2100.0,
                               -1.0 / 40.0};

// Reset the adaptive state of every trajectory: t = t0 + step0 dt, h = dt.
__global__ void k_dp5_reset(const TrajDev* __restrict__ trajs, const AdaptDev* __restrict__ ads, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const TrajDev& T = trajs[i];
    ads[i].st[0] = T.t0 + (double)T.step_base * T.dt;
    ads[i].st[1] = T.dt;
    for (int k = 0; k < 4; ++k) ads[i].cnt[k] = 0;
  }
}

template <int KP, bool ROT, int MK = 0, bool SPLIT = false>
__device__ __forceinline__ void dp5_body(const TrajDev& T, const AdaptDev& A, int prologue, int64_t step0,
                                         int64_t nchunk, int part = 0) {
  extern __shared__ double2 lds[];
  __shared__ double s_red[kTW / 64];
  __shared__ int s_flag;
  __shared__ int s_ok;
  __shared__ double s_nt[kMaxDq * kMaxDq];
  __shared__ double2 s_ph[2 * kMaxDq + 3];
  constexpr bool NM = MK == 2;  // normal-mode model: the layer window and Gram terms of packed_body
  constexpr int NTILE = NM ? 9 : 4;
  const int tid = threadIdx.x;
  const int M = T.M, MM = M * M, L = T.L, d_f = T.d_f, d_q = T.d_q, d_r = T.d_r;
  const int LM = L * M, CT = (NM ? 4 : 3) * M;
  const size_t NM_ = (size_t)T.N * M;
  const double sk = sqrt(T.kappa), sg = sqrt(T.gamma);
  const int areg = (NM ? 7 : 3) * MM;
  double2* St = lds;                               // Gram terms as formed (M x CT)
  double2* Aug = NM ? lds + 4 * MM : lds;          // M x 3M elimination
  double2* Ot = lds + (NM ? 7 : 3) * LM;           // output layer r (kind 2: and r - 1 in Op)
  double2* Op = lds + 8 * LM;
  double2* Wl = lds + (NTILE * LM > areg ? NTILE * LM : areg);
  double* s_drv = reinterpret_cast<double*>(Wl + 2 * MM);  // drive value and frame phases of the pass
  double2* s_prow = Wl + 2 * MM + 10 * kTDriveWin;
  double2* hd = s_prow + 3 * M;
  double* coef = reinterpret_cast<double*>(hd + L);
  double* sq = coef + 3 * L;
  g_double2* gBb = (g_double2*)T.Bb;

  if (tid == 0) s_flag = *T.status;
  for (int rl = tid; rl < L; rl += kTW) {
    const int q = rl / d_f, f = rl - q * d_f;
    const double eq = MK >= 1 ? T.Et[q] - (ROT ? T.w_d * q : 0.0) : T.w_q * q + 0.5 * T.alpha * q * (q - 1);
    const double ff = NM ? T.nm[0] * T.nm[0] * (f + 1 < d_f ? f + 1.0 : 0.0) + T.nm[3] * T.nm[3] * f : (double)f;
    hd[rl] = make_double2(eq + T.w_f * f, -0.5 * (T.kappa * ff + T.gamma * q));
    coef[rl] = 1.0;
    coef[L + rl] = (f + 1 < d_f) ? sk * sqrt((double)(f + 1)) : 0.0;
    coef[2 * L + rl] = (q + 1 < d_q) ? sg * sqrt((double)(q + 1)) : 0.0;
  }
  for (int k = tid; k <= max(max(d_q, d_r), d_f); k += kTW) sq[k] = sqrt((double)k);
  if constexpr (MK >= 1)
    for (int i = tid; i < d_q * d_q; i += kTW) s_nt[i] = T.ntq[i];
  __syncthreads();
  if (s_flag != 0) return;
  if (!prologue && step0 >= T.nsteps) return;
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

  const int NGe = kTW / M;
  const int ej = tid % M, eg = tid / M;
  const bool eact = eg < NGe;
  const int NGp = kTW / CT, KPe = packed_kpe(M, CT);
  const int pc = tid % CT, pg = tid / CT, pi0 = pg * KPe;
  const bool pact = pg < NGp && pi0 < M;
  const int pkind = pc / M, pcc = pc - pkind * M;
  const PackedMap PM{M, CT, L, d_f, KPe, pc, pi0, pkind, pcc, pact};
  double2 acc[KP];
  auto zero_terms = [&]() {
#pragma unroll
    for (int k = 0; k < KP; ++k) acc[k] = make_double2(0.0, 0.0);
  };
  // Gram terms of the output layer r in Ot (kind 2: and of the pair (Op, Ot)), then (kind 2) the
  // output tiles swap so that Op holds layer r
  auto add_terms = [&](int r) {
    packed_terms<KP>(acc, PM, Ot, coef);
    if constexpr (NM) {
      if (r > r_lo) packed_terms_q<KP>(acc, PM, Ot, Op, sk * sq[r]);
    }
  };
  auto swap_out = [&]() {
    if constexpr (NM) {
      double2* t = Ot;
      Ot = Op;
      Op = t;
    }
  };
  // split trajectories: the Gram terms of the parts summed into every part (kind 2: with the pair
  // across the upper boundary, its upper layer read from `upper`, after the part above has
  // published it when `wait`); 0 or -8 (LR_ERR_TIMEOUT)
  auto split_terms = [&](const g_double2* upper, bool wait) -> int {
    if constexpr (SPLIT) {
      if constexpr (NM) {
        if (r_hi < d_r) {
          __syncthreads();
          if (wait && !split_wait_above(T, SS, &s_ok)) return -8;
          double2* const w1[1] = {Ot};
          split_load_layers<1>(w1, upper, r_hi, d_r, LM);
          __syncthreads();
          packed_terms_q<KP>(acc, PM, Ot, Op, sk * sq[r_hi]);
        }
      }
      if (!split_sum<KP>(T, acc, PM, SS, &s_ok)) return -8;
    }
    return 0;
  };
  // W_k of the state whose Gram terms the threads hold, for a right-hand side at time t_use
  auto solve = [&](bool want_fro2, double* fro2, double t_use) -> int {
    if constexpr (NM) {
      const int rc = packed_store<KP>(acc, PM, St, s_red, &s_flag, want_fro2, fro2);
      if (rc) return rc;
      packed_form_c1(St, Aug, M, T.nm, ROT ? frame_phase(T.w_d, t_use) : make_double2(1.0, 0.0));
      return packed_eliminate(Aug, Wl, s_prow, M);
    } else {
      return packed_solve<KP>(acc, PM, Aug, Wl, s_prow, s_red, &s_flag, want_fro2, fro2);
    }
  };
  auto jump_tile = [&](double2* dst, const double2* ym, const double2* y0, const double2* yp, int r, double2 e1j) {
    for (int e = tid; e < LM; e += kTW) {
      const int rl = e / M, j = e - rl * M;
      dst[e] = packed_jump_nm(T, ym, y0, yp, sq, r, rl, rl % d_f, j, e1j);
    }
  };

  // Gram terms and W of the state in `src` (and optional copy to dst), W for time t_use; fro2 of it
  auto gram_pass = [&](const g_double2* src, g_double2* dst, double* fro2, double t_use) -> int {
    zero_terms();
    for (int r = r_lo; r < r_hi; ++r) {
      __syncthreads();
      for (int e = tid; e < LM; e += kTW) {
        const double2 v = ldS(src + (size_t)r * LM + e);
        Ot[e] = v;
        if (dst) stS(dst + (size_t)r * LM + e, v);
      }
      __syncthreads();
      add_terms(r);
      swap_out();
    }
    if (const int rs = split_terms(src, false)) return rs;
    return solve(fro2 != nullptr, fro2, t_use);
  };

  if (!SPLIT && prologue) {  // Gram of the initial state for its observation record
    double f2 = 0.0;
    const int rc = gram_pass(gBb, nullptr, &f2, A.st[0]);
    if (rc) {
      if (tid == 0) report(T, rc, 0);
      return;
    }
    if (tid == 0) {
      *T.fro2 = f2;
      *T.step = 0;
    }
    return;
  }

  // the trajectory's next record time at or after the launch's end: its steps land on its own record
  // times only, whatever the strides of the other trajectories of the batch (which set the launches)
  const int64_t st = T.obs_stride, n_launch = min(step0 + nchunk, T.nsteps);
  const int64_t n_end = st > 0 ? min(T.nsteps, (n_launch + st - 1) / st * st) : T.nsteps;
  const double t_end = T.t0 + (double)(T.step_base + n_end) * T.dt;
  double t = A.st[0], h = A.st[1];
  const bool moves = t < t_end;  // false: an earlier launch has already reached t_end
  int64_t nacc = A.cnt[0], nrej = A.cnt[1];
  int k1slot = (int)A.cnt[2];
  int k1valid = (int)A.cnt[3];
  g_double2* gS[2] = {(g_double2*)T.S0, (g_double2*)T.S1};
  auto Kbuf = [&](int slot) { return (g_double2*)(A.K + (size_t)slot * NM_); };
  const g_double2* ysrc = gBb;  // where y lives (B_n, or the accepted Y_7 until copied)
  int code = 0;

  // One pass: k = f(ts, Y) with Y = `in` (W of Y in Wl), k stored to slot
  // kslot[s - 1]; mode s < 7: Y_{s+1} = y + hc sum_{j <= s} a_{s+1,j} k_j to out,
  // with its Gram terms and W (for the next pass's time t_next); s == 7: the error sum.
  auto stage_pass = [&](int s, double ts, double hc, const g_double2* in, g_double2* out, const int* kslot,
                        double* errsum, double t_next) -> int {
    __syncthreads();
    if (tid == 0) {
      s_drv[0] = drive_at(T, ts);
      const double2 p1 = frame_phase(T.w_d, ts), p2 = frame_phase(2.0 * T.w_d, ts);
      s_drv[1] = p1.x;
      s_drv[2] = p1.y;
      s_drv[3] = p2.x;
      s_drv[4] = p2.y;
    }
    if constexpr (MK >= 1 && ROT)
      if (tid < 2 * d_q + 3) s_ph[tid] = frame_phase((tid - d_q - 1) * T.w_d, ts);
    double2 *Ym2, *Yp, *Yc, *Yn, *Yp2, *Y1c, *Y1n;
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
      Ym2 = Yp2 = Y1c = Y1n = lds;
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
    if constexpr (SPLIT)
      if (s < 7) ++SS.c;
    __syncthreads();
    const double drv = s_drv[0];
    const double2 e1 = make_double2(s_drv[1], s_drv[2]), e2 = make_double2(s_drv[3], s_drv[4]);
    const double2 e1j = ROT ? e1 : make_double2(1.0, 0.0);  // phase of the kind-2 filter jump
    if constexpr (NM) {
      jump_tile(Y1c, Yp, Yc, Yn, r_lo, e1j);
      __syncthreads();
    }
    g_double2* kout = Kbuf(kslot[s - 1]);
    double es = 0.0;
    zero_terms();
    for (int r = r_lo; r < r_hi; ++r) {
      const double him = NM ? -0.5 * T.kappa *
                                  (T.nm[1] * T.nm[1] * (r + 1 < d_r ? r + 1.0 : 0.0) + T.nm[2] * T.nm[2] * r)
                            : 0.0;
      if (eact) {
        const double2* A1 = NM ? Y1c : Yc;  // source tile of the filter jump rows
        for (int rb = eg; rb < L; rb += kTRowBlock * NGe) {
          double2 a1[kTRowBlock], a2[kTRowBlock];
          int s1[kTRowBlock], s2[kTRowBlock];
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
              st_g(kout + gi, kk);  // the stage derivatives' rows are the part's own
              if (s < 7) {
                double2 sum = cscale(kDpA[s][s - 1], kk);
                for (int j = 0; j < s - 1; ++j)
                  if (kDpA[s][j] != 0.0) sum = cfma(kDpA[s][j], ld_g(Kbuf(kslot[j]) + gi), sum);
                const double2 o = cfma(hc, sum, ldS(ysrc + gi));
                stS(out + gi, o);
                Ot[rl * M + ej] = o;
              } else {
                double2 ev = cscale(kDpE[6], kk);
                for (int j = 0; j < 6; ++j)
                  if (kDpE[j] != 0.0) ev = cfma(kDpE[j], ld_g(Kbuf(kslot[j]) + gi), ev);
                const double2 yo = ldS(ysrc + gi), yn = Yc[rl * M + ej];
                const double sc = A.atol + A.rtol * fmax(sqrt(yo.x * yo.x + yo.y * yo.y), sqrt(yn.x * yn.x + yn.y * yn.y));
                const double ex = hc * ev.x / sc, ey = hc * ev.y / sc;
                es += ex * ex + ey * ey;
              }
            }
          }
        }
      }
      __syncthreads();
      if constexpr (SPLIT && NM)
        if (s < 7 && r == r_lo) split_publish_first(T, SS);
      // the next input layer (r + 2; kind 2: r + 3) replaces the oldest one; kind 2 also forms the
      // filter jump of layer r + 1
      const int rnx = NM ? r + 3 : r + 2;
      double2* dstl = NM ? Ym2 : Yp;
      if (rnx < (SPLIT ? min(d_r, r_hi + (NM ? 2 : 1)) : d_r)) {
        if constexpr (SPLIT) {
          double2* const w1[1] = {dstl};
          split_load_layers<1>(w1, in, rnx, d_r, LM);
        } else {
          for (int e = tid; e < LM; e += kTW) dstl[e] = ld_g(in + (size_t)rnx * LM + e);
        }
      }
      if constexpr (NM)
        if (r + 1 < r_hi) jump_tile(Y1n, Yc, Yn, Yp2, r + 1, e1j);
      if (s < 7) add_terms(r);
      __syncthreads();
      if constexpr (NM) {
        double2* tq = Ym2;
        Ym2 = Yp;
        Yp = Yc;
        Yc = Yn;
        Yn = Yp2;
        Yp2 = tq;
        tq = Y1c;
        Y1c = Y1n;
        Y1n = tq;
        swap_out();
      } else {
        double2* tp = Yp;
        Yp = Yc;
        Yc = Yn;
        Yn = tp;
      }
    }
    if (s == 7) {  // fixed-order workgroup sum
      for (int off = 32; off > 0; off >>= 1) es += __shfl_xor(es, off);
      if ((tid & 63) == 0) s_red[tid >> 6] = es;
      __syncthreads();
      double tot = 0.0;
      for (int w = 0; w < kTW / 64; ++w) tot += s_red[w];
      __syncthreads();
      if constexpr (SPLIT)
        if (!split_sum_value(T, tot, &tot, SS, &s_ok)) return -8;
      *errsum = tot;
      return 0;
    }
    if (const int rs = split_terms(out, true)) return rs;
    return solve(false, nullptr, t_next);
  };

  int64_t attempts = 0;
  while (t < t_end) {
    const double hc = fmin(h, t_end - t);
    const bool last = hc >= t_end - t;
    if (!(hc > 1e-14 * fmax(1.0, fabs(t))) || ++attempts > (1 << 22)) {
      code = -9;  // LR_ERR_STEP
      break;
    }
    int kslot[7] = {k1slot, 1, 2, 3, 4, 5, 6 - k1slot};
    if (!k1valid) {
      int rc = gram_pass(gBb, nullptr, nullptr, t);
      if (!rc) rc = stage_pass(1, t, hc, gBb, gS[0], kslot, nullptr, t + kDpC[1] * hc);
      if (rc) {
        code = rc;
        break;
      }
      k1valid = 1;
    } else {  // Y_2 from the stored k_1 (y copied to B_n when it sits in a stage buffer)
      const g_double2* k1 = Kbuf(k1slot);
      const bool copy = ysrc != gBb;
      zero_terms();
      if constexpr (NM) {
        Ot = lds + 7 * LM;
        Op = lds + 8 * LM;
      }
      if constexpr (SPLIT) ++SS.c;
      for (int r = r_lo; r < r_hi; ++r) {
        __syncthreads();
        for (int e = tid; e < LM; e += kTW) {
          const size_t gi = (size_t)r * LM + e;
          const double2 y = ldS(ysrc + gi);
          if (copy) stS(gBb + gi, y);
          const double2 o = cfma(hc * kDpA[1][0], ld_g(k1 + gi), y);
          stS(gS[0] + gi, o);
          Ot[e] = o;
        }
        __syncthreads();
        if constexpr (SPLIT && NM)
          if (r == r_lo) split_publish_first(T, SS);
        add_terms(r);
        swap_out();
      }
      ysrc = gBb;
      int rc = split_terms(gS[0], true);
      if (!rc) rc = solve(false, nullptr, t + kDpC[1] * hc);
      if (rc) {
        code = rc;
        break;
      }
    }
    int rc = 0;
    // stage inputs alternate: Y_2, Y_4, Y_6 in S0; Y_3, Y_5, Y_7 in S1
    for (int s = 2; s <= 6 && !rc; ++s)
      rc = stage_pass(s, t + kDpC[s - 1] * hc, hc, gS[s & 1], gS[(s + 1) & 1], kslot, nullptr, t + kDpC[s] * hc);
    double es = 0.0;
    if (!rc) rc = stage_pass(7, t + hc, hc, gS[1], nullptr, kslot, &es, t + hc);
    if (rc) {
      code = rc;
      break;
    }
    const double err = sqrt(es / (double)NM_);
    if (err <= 1.0) {
      t = last ? t_end : t + hc;
      ++nacc;
      const double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
      if (!(last && hc < h)) h = hc * fac;
      k1slot = 6 - k1slot;
      ysrc = gS[1];
    } else {
      ++nrej;
      h = isfinite(err) ? hc * fmin(1.0, fmax(0.2, 0.9 * pow(err, -0.2))) : hc * 0.2;
    }
  }
  // the state back in B_n, its Gram for the record
  double f2 = 0.0;
  if constexpr (NM) {
    Ot = lds + 7 * LM;
    Op = lds + 8 * LM;
  }
  const int rc = (code || !moves) ? 0 : gram_pass(ysrc, ysrc != gBb ? gBb : nullptr, &f2, t);
  if (tid == 0 && (code || rc)) report(T, code ? code : rc, step0);
  if (tid == 0 && (!SPLIT || part == 0)) {
    A.st[0] = t;
    A.st[1] = h;
    A.cnt[0] = nacc;
    A.cnt[1] = nrej;
    A.cnt[2] = k1slot;
    A.cnt[3] = k1valid;
    if (!code && !rc && moves) *T.fro2 = f2;
    *T.step = n_end;
  }
}

template <int KP>
__global__ __launch_bounds__(kTW) void k_dp5(const TrajDev* __restrict__ trajs, const AdaptDev* __restrict__ ads,
                                             int64_t step0, int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.mkind == 1) {
    if (T.frame)
      dp5_body<KP, true, 1>(T, ads[blockIdx.x], 0, step0, nchunk);
    else
      dp5_body<KP, false, 1>(T, ads[blockIdx.x], 0, step0, nchunk);
  } else if (T.frame) {
    dp5_body<KP, true>(T, ads[blockIdx.x], 0, step0, nchunk);
  } else {
    dp5_body<KP, false>(T, ads[blockIdx.x], 0, step0, nchunk);
  }
}
template <int KP>
__global__ __launch_bounds__(kTW) void k_dp5_prologue(const TrajDev* __restrict__ trajs,
                                                      const AdaptDev* __restrict__ ads, int64_t step0,
                                                      int64_t nchunk) {
  dp5_body<KP, false>(trajs[blockIdx.x], ads[blockIdx.x], 1, step0, nchunk);
}
// The normal-mode model (its own kernels, as in the fixed-step schedule).
template <int KP>
__global__ __launch_bounds__(kTW, (KP <= 8 ? 2 : 1)) void k_dp5_nm(const TrajDev* __restrict__ trajs,
                                                                   const AdaptDev* __restrict__ ads, int64_t step0,
                                                                   int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.frame)
    dp5_body<KP, true, 2>(T, ads[blockIdx.x], 0, step0, nchunk);
  else
    dp5_body<KP, false, 2>(T, ads[blockIdx.x], 0, step0, nchunk);
}
template <int KP>
__global__ __launch_bounds__(kTW, (KP <= 8 ? 2 : 1)) void k_dp5_nm_prologue(const TrajDev* __restrict__ trajs,
                                                                            const AdaptDev* __restrict__ ads,
                                                                            int64_t step0, int64_t nchunk) {
  const TrajDev& T = trajs[blockIdx.x];
  if (T.frame)
    dp5_body<KP, true, 2>(T, ads[blockIdx.x], 1, step0, nchunk);
  else
    dp5_body<KP, false, 2>(T, ads[blockIdx.x], 1, step0, nchunk);
}

// Layer-split trajectories (blockIdx.x -> (trajectory, part) by the tile map;
// chunks only: the prologue is the one-workgroup kernel).
template <int KP>
__global__ __launch_bounds__(kTW) void k_dp5_split(const TrajDev* __restrict__ trajs,
                                                   const AdaptDev* __restrict__ ads, const int2* __restrict__ tilemap,
                                                   int64_t step0, int64_t nchunk) {
  const int2 tw = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tw.x];
  const AdaptDev& A = ads[tw.x];
  if (T.mkind == 1) {
    if (T.frame)
      dp5_body<KP, true, 1, true>(T, A, 0, step0, nchunk, tw.y);
    else
      dp5_body<KP, false, 1, true>(T, A, 0, step0, nchunk, tw.y);
  } else if (T.frame) {
    dp5_body<KP, true, 0, true>(T, A, 0, step0, nchunk, tw.y);
  } else {
    dp5_body<KP, false, 0, true>(T, A, 0, step0, nchunk, tw.y);
  }
}
template <int KP>
__global__ __launch_bounds__(kTW) void k_dp5_split_nm(const TrajDev* __restrict__ trajs,
                                                      const AdaptDev* __restrict__ ads,
                                                      const int2* __restrict__ tilemap, int64_t step0,
                                                      int64_t nchunk) {
  const int2 tw = tilemap[blockIdx.x];
  const TrajDev& T = trajs[tw.x];
  if (T.frame)
    dp5_body<KP, true, 2, true>(T, ads[tw.x], 0, step0, nchunk, tw.y);
  else
    dp5_body<KP, false, 2, true>(T, ads[tw.x], 0, step0, nchunk, tw.y);
}
template <int I = 0>
inline const void* dp5_split_kernel(int kp, bool nm) {
  if constexpr (I + 1 < (int)(sizeof(kPackedKP) / sizeof(int))) {
    if (kp > kPackedKP[I]) return dp5_split_kernel<I + 1>(kp, nm);
  }
  return nm ? (const void*)k_dp5_split_nm<kPackedKP[I]> : (const void*)k_dp5_split<kPackedKP[I]>;
}

template <int I = 0>
inline const void* dp5_kernel(int kp, bool prologue, bool nm = false) {
  if constexpr (I + 1 < (int)(sizeof(kPackedKP) / sizeof(int))) {
    if (kp > kPackedKP[I]) return dp5_kernel<I + 1>(kp, prologue, nm);
  }
  if (nm) return prologue ? (const void*)k_dp5_nm_prologue<kPackedKP[I]> : (const void*)k_dp5_nm<kPackedKP[I]>;
  return prologue ? (const void*)k_dp5_prologue<kPackedKP[I]> : (const void*)k_dp5<kPackedKP[I]>;
}

}  // namespace lrk
