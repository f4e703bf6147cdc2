// Device kernels of the local-relaxation message-passing step for gfx950 (CDNA4).
//
// One pass over a bucket of clusters of dimension De computes, per cluster e
// (paper Sec. 4.2: theta_e, Q_C, Q_{C,beta} and their (sub)gradients):
//   a1  eta = (1 - theta) nu + theta zeta           (Algorithm 2 extrapolation, fused in the loads)
//   a2  theta_e = h_e - sum_children 1 (x) eta_{e->f} + sum_parents eta_{g->e}
//   a3  cyclic Jacobi eigen-decomposition theta_e = U diag(l) U^H
//   a4  Gibbs state rho = U softmax(-beta l) U^H and F_beta (stable shifted form), or the
//       normalised ground projector P0/g and lambda_min
//   a5  partial traces T_{e->f} = Tr_{e\f} rho for every child f, and rho itself when e
//       has parents (consumed by the message update)
//   a8  in certify mode: FP64 lambda_min and the backward-error margin 8 De eps ||theta||_F
// The message kernel applies a6 (gradient and update) per message.
//
// Two cluster kernels:
//   * k_cluster_reg: one lane per cluster, the whole De x De problem in registers with
//     compile-time indexing (De <= 4: sites and edges of 2-local problems).  No LDS, no
//     cross-lane traffic; a wave advances 64 independent clusters.
//   * k_cluster_lds: one wavefront per cluster for 8 <= De <= 64; the matrix lives in LDS and
//     the De/2 disjoint rotations of each round-robin step are applied in parallel.
#pragma once

#include "lrh_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>
#include <utility>

namespace lrh {

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------

// FP32 iterations use the single hardware instructions (v_sqrt_f32, v_rsq_f32, v_rcp_f32,
// v_exp_f32, v_log_f32; about 1 ulp), far inside the FP32 tolerances and much shorter than the
// correctly rounded sequences on the serial chain of a one-lane-per-cluster kernel.  FP64 keeps
// IEEE division, square root and the libm exponential and logarithm.
template <typename T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T drsq(T x);   // 1 / sqrt(x)
template <> __device__ __forceinline__ float drsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double drsq<double>(double x) { return 1.0 / sqrt(x); }
template <typename T> __device__ __forceinline__ T ddiv(T a, T b);   // a / b
template <> __device__ __forceinline__ float ddiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
template <> __device__ __forceinline__ double ddiv<double>(double a, double b) { return a / b; }
template <typename T> __device__ __forceinline__ T dexp(T x);
template <> __device__ __forceinline__ float dexp<float>(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}
template <> __device__ __forceinline__ double dexp<double>(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T dlog(T x);
template <> __device__ __forceinline__ float dlog<float>(float x) {
  return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
}
template <> __device__ __forceinline__ double dlog<double>(double x) { return log(x); }
template <typename T> __device__ __forceinline__ T dfma(T a, T b, T c);
template <> __device__ __forceinline__ float dfma<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ __forceinline__ double dfma<double>(double a, double b, double c) { return fma(a, b, c); }

// Algorithm 2 extrapolation / averaging (1 - th) x + th y, with one explicit rounding
// pattern so that every kernel computing it from the same inputs gets the same bits.
// Cluster handled by workgroup i of a launch with one workgroup per cluster (n of them).  The
// dispatcher hands consecutive workgroups to the 8 XCDs in turn, and each XCD has its own L2;
// consecutive clusters read neighbouring messages (one cache line holds the same component of
// many consecutive messages), so every XCD takes one contiguous run of clusters instead.
__device__ __forceinline__ int64_t xcd_cluster(int64_t i, int64_t n) {
  constexpr int64_t kXcd = 8;
  const int64_t q = n / kXcd, r = n % kXcd;
  const int64_t x = i % kXcd, j = i / kXcd;
  return x * q + (x < r ? x : r) + j;
}

template <typename T>
__device__ __forceinline__ T extrap(T x, T y, T th) {
  return dfma<T>(T(1) - th, x, th * y);
}

// Jacobi rotation parameters for a pair with (real-ified) off-diagonal magnitude r > 0:
// tau = (a_qq - a_pp) / (2 r), t = sign(tau) / (|tau| + sqrt(tau^2 + 1)), c = 1/sqrt(1+t^2).
template <typename T>
__device__ __forceinline__ void rot_params(T app, T aqq, T r, T& t, T& c, T& s) {
  T tau = ddiv<T>(aqq - app, T(2) * r);
  T at = fabs(tau);
  t = ddiv<T>(tau >= T(0) ? T(1) : T(-1), at + dsqrt<T>(dfma<T>(tau, tau, T(1))));
  c = drsq<T>(dfma<T>(t, t, T(1)));
  s = t * c;
}

__host__ __device__ constexpr int pdep_bits(int a, int x, int mask, int nbits) {
  int out = 0, ia = 0, ix = 0;
  for (int b = 0; b < nbits; ++b) {
    if ((mask >> b) & 1) { out |= ((a >> ia) & 1) << b; ++ia; }
    else { out |= ((x >> ix) & 1) << b; ++ix; }
  }
  return out;
}
__host__ __device__ constexpr int pext_bits(int i, int mask, int nbits) {
  int out = 0, k = 0;
  for (int b = 0; b < nbits; ++b)
    if ((mask >> b) & 1) { out |= ((i >> b) & 1) << k; ++k; }
  return out;
}
__host__ __device__ constexpr int log2i(int D) { return D <= 1 ? 0 : 1 + log2i(D / 2); }

// ------------------------------------------------------------------------------------------
// register-resident cluster kernel (one lane per cluster, D_e <= 8)
// ------------------------------------------------------------------------------------------

// Hermitian D x D matrix kept as its packed upper triangle (real parts and imaginary parts);
// every index is a compile-time constant after unrolling, so the storage lives in registers
// and each independent entry is carried once across the sweep loop.
template <typename T, bool CPLX, int D>
struct HMat {
  static constexpr int NT = D * (D + 1) / 2;
  T r[NT];
  T i[CPLX ? NT : 1];
  __device__ __forceinline__ T re(int a, int b) const {
    return a <= b ? r[tri_index(a, b, D)] : r[tri_index(b, a, D)];
  }
  __device__ __forceinline__ T im(int a, int b) const {
    if constexpr (!CPLX) return T(0);
    else return a < b ? i[tri_index(a, b, D)] : (a > b ? -i[tri_index(b, a, D)] : T(0));
  }
  __device__ __forceinline__ void set(int a, int b, T vr, T vi) {
    if (a <= b) {
      r[tri_index(a, b, D)] = vr;
      if constexpr (CPLX) i[tri_index(a, b, D)] = (a == b) ? T(0) : vi;
    } else {
      r[tri_index(b, a, D)] = vr;
      if constexpr (CPLX) i[tri_index(b, a, D)] = -vi;
    }
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      r[k] = T(0);
      if constexpr (CPLX) i[k] = T(0);
    }
  }
};

// packed message / term components <-> HMat (layout: real upper triangle row-major, then the
// imaginary strict upper triangle)
template <typename T, bool CPLX, int D, typename Get>
__device__ __forceinline__ void unpack(Get get, HMat<T, CPLX, D>& M) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) M.r[tri_index(a, b, D)] = get(tri_index(a, b, D));
  if constexpr (CPLX) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      M.i[tri_index(a, a, D)] = T(0);
#pragma unroll
      for (int b = a + 1; b < D; ++b) M.i[tri_index(a, b, D)] = get(D * (D + 1) / 2 + stri_index(a, b, D));
    }
  }
}

template <typename T, bool CPLX, int D, typename Get>
__device__ __forceinline__ void unpack_add(Get get, HMat<T, CPLX, D>& M) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) M.r[tri_index(a, b, D)] += get(tri_index(a, b, D));
  if constexpr (CPLX) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) M.i[tri_index(a, b, D)] += get(D * (D + 1) / 2 + stri_index(a, b, D));
  }
}

template <typename T, bool CPLX, int D, typename Put>
__device__ __forceinline__ void pack(Put put, const HMat<T, CPLX, D>& M) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) put(tri_index(a, b, D), M.r[tri_index(a, b, D)]);
  if constexpr (CPLX) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) put(D * (D + 1) / 2 + stri_index(a, b, D), M.i[tri_index(a, b, D)]);
  }
}

// Calls f(integral_constant<int, M>) for the compile-time mask M == mask among the masks that
// select log2(DC) of the log2(DE) site bits (the positions a child can occupy in its parent).
// A flat fold over the candidate masks (no recursion), so everything inlines into the caller.
template <int DE, int DC, int M, typename F>
__device__ __forceinline__ void mask_case(int mask, F& f) {
  if constexpr (__builtin_popcount(M) == log2i(DC)) {
    if (mask == M) {
      f(std::integral_constant<int, M>{});
      // An empty statement that differs per case: without it the compiler merges the cases into
      // one path that indexes the register matrices with a runtime offset, which moves them to
      // scratch memory (12-24 bytes per lane in every register kernel with children).
      __asm__ volatile("; mask case %0" :: "n"(M));
    }
  }
}
template <int DE, int DC, typename F, int... I>
__device__ __forceinline__ void mask_dispatch_seq(int mask, F& f, std::integer_sequence<int, I...>) {
  (mask_case<DE, DC, I + 1>(mask, f), ...);
}
template <int DE, int DC, typename F>
__device__ __forceinline__ void mask_dispatch(int mask, F&& f) {
  mask_dispatch_seq<DE, DC>(mask, f, std::make_integer_sequence<int, DE - 1>{});
}

// theta_e -= 1_{e\f} (x) X for a child whose sites occupy bit mask MASK of e's index.
template <typename T, bool CPLX, int DE, int DC, int MASK>
__device__ __forceinline__ void lift_sub(HMat<T, CPLX, DE>& A, const HMat<T, CPLX, DC>& X) {
  constexpr int NB = log2i(DE);
#pragma unroll
  for (int a = 0; a < DE; ++a)
#pragma unroll
    for (int b = a; b < DE; ++b) {
      if (((a ^ b) & ~MASK & (DE - 1)) == 0) {
        const int x = pext_bits(a, MASK, NB), y = pext_bits(b, MASK, NB);
        A.r[tri_index(a, b, DE)] -= X.re(x, y);
        if constexpr (CPLX) A.i[tri_index(a, b, DE)] -= X.im(x, y);
      }
    }
}

// T = Tr_{e\f} rho for a child at mask MASK.
template <typename T, bool CPLX, int DE, int DC, int MASK>
__device__ __forceinline__ void ptrace_reg(const HMat<T, CPLX, DE>& Rh, HMat<T, CPLX, DC>& Tm) {
  constexpr int NB = log2i(DE);
  constexpr int NR = DE / DC;
#pragma unroll
  for (int a = 0; a < DC; ++a)
#pragma unroll
    for (int b = a; b < DC; ++b) {
      T sr = T(0), si = T(0);
#pragma unroll
      for (int x = 0; x < NR; ++x) {
        sr += Rh.re(pdep_bits(a, x, MASK, NB), pdep_bits(b, x, MASK, NB));
        if constexpr (CPLX) si += Rh.im(pdep_bits(a, x, MASK, NB), pdep_bits(b, x, MASK, NB));
      }
      Tm.set(a, b, sr, si);
    }
}

// One cyclic sweep of two-sided Jacobi rotations over all pairs (p < q), row-cyclic order.
// Branch-free: a pair with a_pq == 0 gets the identity rotation (t = 0, c = 1, s = 0), so the
// unrolled sweep is straight-line code.
template <typename T, bool CPLX, int D, bool VEC>
__device__ __forceinline__ void jacobi_sweep_reg(HMat<T, CPLX, D>& A, T (&ur)[D][D], T (&ui)[D][D]) {
#pragma unroll
  for (int p = 0; p < D - 1; ++p)
#pragma unroll
    for (int q = p + 1; q < D; ++q) {
      const T xr = A.re(p, q);
      const T xi = A.im(p, q);
      const T r = CPLX ? dsqrt<T>(dfma<T>(xr, xr, xi * xi)) : fabs(xr);
      const bool nz = (r != T(0));
      const T rs = nz ? r : T(1);
      // e^{-i phi} with a_pq = r e^{i phi}; real case: sign(a_pq)
      T er, ei;
      if constexpr (CPLX) {
        er = nz ? ddiv<T>(xr, rs) : T(1);
        ei = nz ? ddiv<T>(-xi, rs) : T(0);
      } else {
        er = nz ? copysign(T(1), xr) : T(1);
        ei = T(0);
      }
      const T app = A.re(p, p), aqq = A.re(q, q);
      T t, c, s;
      rot_params<T>(app, aqq, rs, t, c, s);
      t = nz ? t : T(0);
      c = nz ? c : T(1);
      s = nz ? s : T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if (k == p || k == q) continue;
        // column update (A G): w = a_kq e^{-i phi}; rows follow by Hermitian symmetry
        const T pr = A.re(k, p), pi = A.im(k, p);
        const T qr = A.re(k, q), qi = A.im(k, q);
        const T wr = CPLX ? (qr * er - qi * ei) : qr * er;
        const T wi = CPLX ? (qr * ei + qi * er) : T(0);
        A.set(k, p, c * pr - s * wr, c * pi - s * wi);
        A.set(k, q, s * pr + c * wr, s * pi + c * wi);
      }
      A.set(p, p, app - t * r, T(0));
      A.set(q, q, aqq + t * r, T(0));
      A.set(p, q, nz ? T(0) : xr, nz ? T(0) : xi);
      if constexpr (VEC) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const T pr = ur[k][p], pi = CPLX ? ui[k][p] : T(0);
          const T qr = ur[k][q], qi = CPLX ? ui[k][q] : T(0);
          const T wr = CPLX ? (qr * er - qi * ei) : qr * er;
          const T wi = CPLX ? (qr * ei + qi * er) : T(0);
          ur[k][p] = c * pr - s * wr;
          ur[k][q] = s * pr + c * wr;
          if constexpr (CPLX) {
            ui[k][p] = c * pi - s * wi;
            ui[k][q] = s * pi + c * wi;
          }
        }
      }
    }
}

// Squared off-diagonal Frobenius norm, accumulated in FP64 whatever T: the convergence test of
// the FP32 iterations is taken in FP64, so near-degenerate clusters (large rotation angles on
// tiny off-diagonals) are judged on the FP32 matrix without a second rounding of the test.
template <typename T, bool CPLX, int D>
__device__ __forceinline__ double offdiag2(const HMat<T, CPLX, D>& A) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a + 1; b < D; ++b) {
      const double x = (double)A.r[tri_index(a, b, D)];
      s = fma(x, x, s);
      if constexpr (CPLX) {
        const double y = (double)A.i[tri_index(a, b, D)];
        s = fma(y, y, s);
      }
    }
  return 2.0 * s;
}

template <typename T>
struct FusedCoef { T thp, ithp, thc; };

// Read in place of an absent coefficient row or term block, so that those loads need no branch.
// 64 doubles hold a packed complex 8 x 8 block, the largest a register kernel takes.
static __device__ FusedParams kZeroRow;
static __device__ double kZeroTerms[64];

template <typename T, bool CPLX, int DE, int DC, int MODE>
__device__ void cluster_reg_body(const ClusterArgs<T>& A, int64_t c) {
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  HMat<T, CPLX, DE> H;
  const bool fused = (A.fp != nullptr);
  // iteration coefficients: the fused row, else the stage table row, else the launch's own
  // theta and beta (fused launches are replayed from a graph across stages)
  const bool from_row = fused || A.tab != nullptr;
  const FusedParams* fq = fused ? A.fp : (A.tab ? A.tab : &kZeroRow);
  const FusedCoef<T> fc{(T)fq->theta_prev, (T)fq->inv_thL_prev, (T)fq->theta_cur};
  const T th = from_row ? fc.thc : (T)A.theta;
  const T beta = from_row ? (T)fq->beta : (T)A.beta;
  // Loads are issued in two waves before any arithmetic or store: first every index (h offset,
  // child and parent message ids, masks, marginal slots), then every value, branch-free with a
  // valid index for an empty slot.  One cluster per lane and a cold L2 make each dependent round
  // trip a full memory latency.  This applies to single-site children (at most log2(D_e) of
  // them) and to the first kHoistPar parents of a 2 x 2 cluster; larger cases keep the plain
  // per-slot loops.  The arithmetic and its order are unchanged.
  constexpr bool HOIST_CH = (DC == 2);
  constexpr bool HOIST_PAR = (DE == 2);
  constexpr int MAXCH = HOIST_CH ? log2i(DE) : 1;
  constexpr int NCC = HOIST_CH ? (CPLX ? 4 : 3) : 1;
  constexpr int NCP = HOIST_PAR ? (CPLX ? 4 : 3) : 1;
  constexpr int kHoistPar = 4;
  // Source pointers are chosen per launch so that every hoisted load below is unconditional: an
  // absent array is replaced by one that is present and the value read from it is never used,
  // and an empty slot reads message 0 (a child or parent bucket that exists holds at least one).
  const bool need_g = fused && !A.fused_first;  // the fused form's gradient step
  // ---- index loads ----
  const int64_t ho = A.hoff[c];
  const int32_t gid = A.gid[c];
  const int32_t rs_read = (A.rslot ? A.rslot : A.gid)[c];  // gid: a stand-in of n entries
  const int64_t rs_self = A.rslot ? rs_read : -1;
  int cm[MAXCH], cmask[MAXCH], crs[MAXCH];
  if constexpr (HOIST_CH) {
    const int32_t* rsp = fused ? A.ch_rslot : A.ch;  // the launcher requires ch_rslot when fused
#pragma unroll
    for (int s = 0; s < MAXCH; ++s) {
      const int64_t so = (int64_t)(s < A.maxch ? s : 0) * A.n + c;
      const int m = A.ch[so];
      cm[s] = s < A.maxch ? m : -1;
      cmask[s] = A.chmask[so];
      crs[s] = rsp[so];
    }
  }
  int pm[kHoistPar];
  if constexpr (HOIST_PAR) {
    if (A.maxpar > 0) {
#pragma unroll
      for (int s = 0; s < kHoistPar; ++s) {
        const int m = A.par[(int64_t)(s < A.maxpar ? s : 0) * A.n + c];
        pm[s] = s < A.maxpar ? m : -1;
      }
    } else {
#pragma unroll
      for (int s = 0; s < kHoistPar; ++s) pm[s] = -1;
    }
  }
  // ---- value loads ----
  static_assert((CPLX ? DE * DE : DE * (DE + 1) / 2) <= 64, "term block beyond kZeroTerms");
  const double* hb = ho >= 0 ? A.h + ho : kZeroTerms;
  unpack<T, CPLX, DE>([&](int k) { return (T)hb[k]; }, H);
  T cn[MAXCH][NCC], cz[MAXCH][NCC], cg[MAXCH][NCC];
  if constexpr (HOIST_CH) {
    const T* sN = fused ? A.nu_c_prev : A.nu_c;
    const T* sZ = fused ? A.ze_c_prev : (A.ze_c ? A.ze_c : A.nu_c);
    const T* sR = need_g ? A.Rprev_c : sN;
    const T* sT = need_g ? A.Tprev_c : sN;
#pragma unroll
    for (int s = 0; s < MAXCH; ++s) {
      const int64_t m = cm[s] >= 0 ? cm[s] : 0;
      const int64_t rs = crs[s] >= 0 ? crs[s] : 0;
#pragma unroll
      for (int k = 0; k < NCC; ++k) {
        const int64_t o = (int64_t)k * A.Mc + m;
        cn[s][k] = sN[o];
        cz[s][k] = sZ[o];
        cg[s][k] = sR[need_g ? (int64_t)k * A.Sc + rs : o] - sT[o];
      }
    }
  }
  T pn[kHoistPar][NCP], pz[kHoistPar][NCP], pg[kHoistPar][NCP];
  if constexpr (HOIST_PAR) {
    if (A.maxpar > 0) {
      const T* sN = fused ? A.nu_p_prev : A.nu_p;
      const T* sZ = fused ? A.ze_p_prev : (A.ze_p ? A.ze_p : A.nu_p);
      const T* sR = need_g ? A.Rprev_p : sN;
      const T* sT = need_g ? A.Tprev_p : sN;
      const int64_t rs = rs_self >= 0 ? rs_self : 0;
      T r[NCP];
#pragma unroll
      for (int k = 0; k < NCP; ++k) r[k] = sR[need_g ? (int64_t)k * A.S + rs : (int64_t)k * A.Mp];
#pragma unroll
      for (int s = 0; s < kHoistPar; ++s) {
        const int64_t m = pm[s] >= 0 ? pm[s] : 0;
#pragma unroll
        for (int k = 0; k < NCP; ++k) {
          const int64_t o = (int64_t)k * A.Mp + m;
          pn[s][k] = sN[o];
          pz[s][k] = sZ[o];
          pg[s][k] = r[k] - sT[o];
        }
      }
    }
  }
  // ---- children: subtract lifted messages ----
  if constexpr (HOIST_CH) {
#pragma unroll
    for (int s = 0; s < MAXCH; ++s) {
      if (cm[s] < 0) continue;
      HMat<T, CPLX, DC> X;
      if (fused) {
        unpack<T, CPLX, DC>([&](int k) {
          T nu0 = cn[s][k], ze0 = cz[s][k];
          if (!A.fused_first) {
            ze0 = dfma<T>(cg[s][k], fc.ithp, ze0);
            nu0 = extrap<T>(nu0, ze0, fc.thp);
            const int64_t o = (int64_t)k * A.Mc + cm[s];
            A.nu_c_new[o] = nu0;
            A.ze_c_new[o] = ze0;
          }
          return extrap<T>(nu0, ze0, th);
        }, X);
      } else if (A.ze_c) {
        unpack<T, CPLX, DC>([&](int k) { return extrap<T>(cn[s][k], cz[s][k], th); }, X);
      } else {
        unpack<T, CPLX, DC>([&](int k) { return cn[s][k]; }, X);
      }
      mask_dispatch<DE, DC>(cmask[s], [&](auto mc) __attribute__((always_inline)) {
        lift_sub<T, CPLX, DE, DC, decltype(mc)::value>(H, X);
      });
    }
  } else if constexpr (DC > 0) {
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int mask = A.chmask[(int64_t)s * A.n + c];
      HMat<T, CPLX, DC> X;
      if (fused) {
        // by (slot, cluster) when available: the same level of dependent loads as ch itself
        const int64_t rs = A.ch_rslot ? A.ch_rslot[(int64_t)s * A.n + c] : A.rslot_of_msg_c[m];
        unpack<T, CPLX, DC>([&](int k) {
          const int64_t o = (int64_t)k * A.Mc + m;
          T nu0 = A.nu_c_prev[o], ze0 = A.ze_c_prev[o];
          if (!A.fused_first) {
            T g = A.Rprev_c[(int64_t)k * A.Sc + rs] - A.Tprev_c[o];
            ze0 = dfma<T>(g, fc.ithp, ze0);
            nu0 = extrap<T>(nu0, ze0, fc.thp);
            A.nu_c_new[o] = nu0;
            A.ze_c_new[o] = ze0;
          }
          return extrap<T>(nu0, ze0, th);
        }, X);
      } else if (A.ze_c) {
        unpack<T, CPLX, DC>([&](int k) {
          const int64_t o = (int64_t)k * A.Mc + m;
          return extrap<T>(A.nu_c[o], A.ze_c[o], th);
        }, X);
      } else {
        unpack<T, CPLX, DC>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, X);
      }
      mask_dispatch<DE, DC>(mask, [&](auto mc) __attribute__((always_inline)) {
        lift_sub<T, CPLX, DE, DC, decltype(mc)::value>(H, X);
      });
    }
  }
  // ---- parents: add messages received ----
  int s_par0 = 0;
  if constexpr (HOIST_PAR) {
#pragma unroll
    for (int s = 0; s < kHoistPar; ++s) {
      if (pm[s] < 0) continue;
      if (fused) {
        unpack_add<T, CPLX, DE>([&](int k) {
          T nu0 = pn[s][k], ze0 = pz[s][k];
          if (!A.fused_first) {
            ze0 = dfma<T>(pg[s][k], fc.ithp, ze0);
            nu0 = extrap<T>(nu0, ze0, fc.thp);
          }
          return extrap<T>(nu0, ze0, th);
        }, H);
      } else if (A.ze_p) {
        unpack_add<T, CPLX, DE>([&](int k) { return extrap<T>(pn[s][k], pz[s][k], th); }, H);
      } else {
        unpack_add<T, CPLX, DE>([&](int k) { return pn[s][k]; }, H);
      }
    }
    s_par0 = kHoistPar;
  }
  for (int s = s_par0; s < A.maxpar; ++s) {
    const int m = A.par[(int64_t)s * A.n + c];
    if (m < 0) continue;
    if (fused) {
      unpack_add<T, CPLX, DE>([&](int k) {
        const int64_t o = (int64_t)k * A.Mp + m;
        T nu0 = A.nu_p_prev[o], ze0 = A.ze_p_prev[o];
        if (!A.fused_first) {
          T g = A.Rprev_p[(int64_t)k * A.S + rs_self] - A.Tprev_p[o];
          ze0 = dfma<T>(g, fc.ithp, ze0);
          nu0 = extrap<T>(nu0, ze0, fc.thp);
        }
        return extrap<T>(nu0, ze0, th);
      }, H);
    } else if (A.ze_p) {
      unpack_add<T, CPLX, DE>([&](int k) {
        const int64_t o = (int64_t)k * A.Mp + m;
        return extrap<T>(A.nu_p[o], A.ze_p[o], th);
      }, H);
    } else {
      unpack_add<T, CPLX, DE>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, H);
    }
  }
  // ---- a3: cyclic Jacobi (norms and the convergence test in FP64) ----
  double dg = 0.0;
#pragma unroll
  for (int k = 0; k < DE; ++k) {
    const double x = (double)H.r[tri_index(k, k, DE)];
    dg = fma(x, x, dg);
  }
  const double nrm2 = dg + offdiag2<T, CPLX, DE>(H);
  T ur[DE][DE], ui[DE][DE];  // eigenvectors (unused, and removed, without VEC / CPLX)
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = 0; j < DE; ++j) {
        ur[i][j] = (i == j) ? T(1) : T(0);
        if constexpr (CPLX) ui[i][j] = T(0);
      }
  }
  const double tol2 = A.tol * A.tol * nrm2;
  bool conv = false;
  for (int sweep = 0; sweep <= A.max_sweeps; ++sweep) {
    if (offdiag2<T, CPLX, DE>(H) <= tol2) { conv = true; break; }
    if (sweep == A.max_sweeps) break;
    if constexpr (VEC) jacobi_sweep_reg<T, CPLX, DE, true>(H, ur, ui);
    else {
      T dr[DE][DE], di[DE][DE];
      jacobi_sweep_reg<T, CPLX, DE, false>(H, dr, di);
    }
  }
  if (!conv && A.noconv) atomicAdd(A.noconv, 1ull);
  T lam[DE];
  T lmin = H.r[0];
#pragma unroll
  for (int k = 0; k < DE; ++k) { lam[k] = H.r[tri_index(k, k, DE)]; lmin = fmin(lmin, lam[k]); }
  if (!isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  if constexpr (MODE == MODE_CERTIFY) {
    // The rotated matrix differs from a diagonal one by its remaining off-diagonal part, so
    // lambda_min >= min diag - ||off||_2 >= min diag - ||off||_F (Weyl): the bound holds whether or
    // not the sweeps reached the tolerance.  The first term is the backward error of the rotations.
    A.scal[gid] = (double)lmin;
    A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt((double)nrm2) + sqrt(offdiag2<T, CPLX, DE>(H));
    return;
  } else {
    // ---- a4: marginal weights ----
    T p[DE];
    if constexpr (MODE == MODE_GIBBS) {
      const T b = beta;
      T Z = T(0);
#pragma unroll
      for (int k = 0; k < DE; ++k) { p[k] = dexp<T>(-b * (lam[k] - lmin)); Z += p[k]; }
      const T iZ = ddiv<T>(T(1), Z);
#pragma unroll
      for (int k = 0; k < DE; ++k) p[k] *= iZ;
      if (A.scal) A.scal[gid] = (double)(lmin - ddiv<T>(dlog<T>(Z), b));
    } else {
      const T tau = (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2));
      T g = T(0);
#pragma unroll
      for (int k = 0; k < DE; ++k) { p[k] = (lam[k] <= lmin + tau) ? T(1) : T(0); g += p[k]; }
      const T ig = ddiv<T>(T(1), g);
#pragma unroll
      for (int k = 0; k < DE; ++k) p[k] *= ig;
      if (A.scal) A.scal[gid] = (double)lmin;
    }
    // rho = U diag(p) U^H  (reuse H)
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = i; j < DE; ++j) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < DE; ++k) {
          const T a_r = ur[i][k] * p[k], a_i = CPLX ? ui[i][k] * p[k] : T(0);
          // (a_r + i a_i) * conj(u_jk)
          sr = dfma<T>(a_r, ur[j][k], sr);
          if constexpr (CPLX) {
            sr = dfma<T>(a_i, ui[j][k], sr);
            si = dfma<T>(a_i, ur[j][k], si);
            si = dfma<T>(-a_r, ui[j][k], si);
          }
        }
        H.set(i, j, sr, si);
      }
    // ---- outputs: own marginal ----
    if (rs_self >= 0 && A.R) {
      pack<T, CPLX, DE>([&](int k, T v) { A.R[(int64_t)k * A.S + rs_self] = v; }, H);
    }
    if (A.marg) {
      T* mo = A.marg + A.marg_off[gid];
      pack<T, CPLX, DE>([&](int k, T v) { mo[k] = v; }, H);
    }
    // ---- a5: partial traces onto the children ----
    if constexpr (DC > 0) {
      if (A.Tout) {
        // (unrolled, so that the hoisted slot arrays are indexed by constants and stay in registers)
#pragma unroll
        for (int s = 0; s < (HOIST_CH ? MAXCH : A.maxch); ++s) {
          int m, mask;
          if constexpr (HOIST_CH) {
            m = cm[s];
            mask = cmask[s];
          } else {
            m = A.ch[(int64_t)s * A.n + c];
            mask = m >= 0 ? A.chmask[(int64_t)s * A.n + c] : 0;
          }
          if (m < 0) continue;
          HMat<T, CPLX, DC> Tm;
          mask_dispatch<DE, DC>(mask, [&](auto mc) __attribute__((always_inline)) {
            ptrace_reg<T, CPLX, DE, DC, decltype(mc)::value>(H, Tm);
          });
          pack<T, CPLX, DC>([&](int k, T v) { A.Tout[(int64_t)k * A.Mc + m] = v; }, Tm);
        }
      }
    }
  }
}

template <typename T, bool CPLX, int DE, int DC, int MODE>
__global__ __launch_bounds__(256) void k_cluster_reg(ClusterArgs<T> A) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < A.n) cluster_reg_body<T, CPLX, DE, DC, MODE>(A, c);
}

// ------------------------------------------------------------------------------------------
// wave-per-cluster LDS kernel (8 <= De <= 64)
// ------------------------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Reductions over the 64 lanes of a wave built from DPP row operations (xor 1, xor 2, mirror
// within 8 lanes, mirror within 16 lanes: every lane of a row of 16 ends with the same sum) and
// four readlanes, instead of six LDS-crossbar shuffles.  Every lane of the wave must be active;
// the result is wave-uniform.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return v;
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = row_sum16(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_min_dpp(double v) {
  v = fmin(v, dpp_mov<0xB1>(v));
  v = fmin(v, dpp_mov<0x4E>(v));
  v = fmin(v, dpp_mov<0x141>(v));
  v = fmin(v, dpp_mov<0x140>(v));
  return fmin(fmin(readlane_d(v, 0), readlane_d(v, 16)), fmin(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_max_rows(double v) {   // v already uniform within each row
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int pdep_rt(int a, int x, int mask, int nbits) {
  int out = 0, ia = 0, ix = 0;
  for (int b = 0; b < nbits; ++b) {
    if ((mask >> b) & 1) { out |= ((a >> ia) & 1) << b; ++ia; }
    else { out |= ((x >> ix) & 1) << b; ++ix; }
  }
  return out;
}
__device__ __forceinline__ int pext_rt(int i, int mask, int nbits) {
  int out = 0, k = 0;
  for (int b = 0; b < nbits; ++b)
    if ((mask >> b) & 1) { out |= ((i >> b) & 1) << k; ++k; }
  return out;
}

// round-robin tournament: round r (0..D-2), pair k (0..D/2-1) -> (p < q); every pair once.
__device__ __forceinline__ void rr_pair(int r, int k, int D, int& p, int& q) {
  if (k == 0) { p = r; q = D - 1; }
  else { p = (r + k) % (D - 1); q = (r - k + (D - 1)) % (D - 1); }
  if (p > q) { int t = p; p = q; q = t; }
}

// element (a, b) of a packed Hermitian stored at stride `st` (component k at base[k*st])
template <typename T, typename Get>
__device__ __forceinline__ void herm_elem(Get get, int a, int b, int D, bool cplx, T& vr, T& vi) {
  if (a <= b) {
    vr = get(tri_index(a, b, D));
    vi = (cplx && a < b) ? get(D * (D + 1) / 2 + stri_index(a, b, D)) : T(0);
  } else {
    vr = get(tri_index(b, a, D));
    vi = cplx ? -get(D * (D + 1) / 2 + stri_index(b, a, D)) : T(0);
  }
}

// Element (a, b) of a packed Hermitian without branches: both addresses are always valid, the
// imaginary part is selected (conjugated below the diagonal, zero on it).
template <typename T, bool CPLX, typename Get>
__device__ __forceinline__ void herm_elem_bf(Get get, int a, int b, int D, T& vr, T& vi) {
  const int lo = min(a, b), hi = max(a, b);
  vr = get(tri_index(lo, hi, D));
  if constexpr (CPLX) {
    const T v = get(D * (D + 1) / 2 + (lo < hi ? stri_index(lo, hi, D) : 0));
    vi = a < b ? v : (a > b ? -v : T(0));
  } else {
    vi = T(0);
  }
}

// ---- shared pieces of the LDS kernels ----
//
// A 64-lane wave holds G = 64/W clusters, W lanes each (W is a power of two, 8..64); lane `lt`
// of a cluster strides over that cluster's entries by W.  Every loop whose trip count depends
// on the data is made wave-uniform (per-cluster `done` flags, exit on __all), so barriers and
// cross-lane shuffles always see the whole wave.

template <int W, typename T>
__device__ __forceinline__ T seg_sum(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int W, typename T>
__device__ __forceinline__ T seg_min(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// theta_e = [h_e] - sum_children 1 (x) x_{e->f} + sum_parents x_{g->e}, written to (dr, di) with
// leading dimension DE+1; x = extrap(nu, zeta, th) when zeta is given.  Off-diagonal message
// elements are scaled by `offs` (packed-coordinate cotangents use 1/2).  Returns this lane's
// share of the squared Frobenius norm.
template <typename T, bool CPLX, int DE, int W>
__device__ T lds_assemble(const ClusterArgs<T>& A, int64_t c, int lt, const T* xc, const T* zc, const T* xp,
                          const T* zp, T th, bool with_h, T offs, T* dr, T* di) {
  constexpr int LD = DE + 1;
  constexpr int NB = log2i(DE);
  const int64_t ho = with_h ? A.hoff[c] : -1;
  const int Dc = A.Dc;
  T my_n2 = T(0);
  for (int idx = lt; idx < DE * DE; idx += W) {
    const int i = idx / DE, j = idx % DE;
    T vr = T(0), vi = T(0);
    if (ho >= 0) {
      const double* h = A.h + ho;
      herm_elem<T>([&](int k) { return (T)h[k]; }, i, j, DE, CPLX, vr, vi);
    }
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int mask = A.chmask[(int64_t)s * A.n + c];
      if (((i ^ j) & ~mask & (DE - 1)) != 0) continue;
      const int a = pext_rt(i, mask, NB), b = pext_rt(j, mask, NB);
      T er, ei;
      if (zc)
        herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mc + m;
                                  return extrap<T>(xc[o], zc[o], th); }, a, b, Dc, CPLX, er, ei);
      else
        herm_elem<T>([&](int k) { return xc[(int64_t)k * A.Mc + m]; }, a, b, Dc, CPLX, er, ei);
      const T sc = (a == b) ? T(1) : offs;
      vr -= sc * er;
      vi -= sc * ei;
    }
    for (int s = 0; s < A.maxpar; ++s) {
      const int m = A.par[(int64_t)s * A.n + c];
      if (m < 0) continue;
      T er, ei;
      if (zp)
        herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mp + m;
                                  return extrap<T>(xp[o], zp[o], th); }, i, j, DE, CPLX, er, ei);
      else
        herm_elem<T>([&](int k) { return xp[(int64_t)k * A.Mp + m]; }, i, j, DE, CPLX, er, ei);
      const T sc = (i == j) ? T(1) : offs;
      vr += sc * er;
      vi += sc * ei;
    }
    dr[i * LD + j] = vr;
    if constexpr (CPLX) di[i * LD + j] = vi;
    my_n2 = dfma<T>(vr, vr, my_n2);
    if constexpr (CPLX) my_n2 = dfma<T>(vi, vi, my_n2);
  }
  return my_n2;
}

// Rotation scratch of the round-robin parallel Jacobi (one per cluster).
template <typename T, int NP>
struct JacobiScratch {
  T c[NP], s[NP], er[NP], ei[NP], app[NP], aqq[NP];
  int p[NP], q[NP];
};

// Cyclic two-sided Jacobi on the LDS matrix (sar, sai) with eigenvectors accumulated in
// (sur, sui) when VEC.  Each round applies the DE/2 disjoint rotations of a round-robin
// tournament in parallel: columns (A G, U G), then rows (G^H A), then the exact 2x2 blocks.
// `done` clusters (converged, capped, or absent) skip the work but keep the wave together.
// Returns true when the off-diagonal norm fell below tol2 within max_sweeps sweeps.
template <typename T, bool CPLX, int DE, bool VEC, int W>
__device__ bool lds_jacobi(T* sar, T* sai, T* sur, T* sui, JacobiScratch<T, DE / 2>& J, double tol2, int max_sweeps,
                           int lt, bool active) {
  constexpr int LD = DE + 1;
  constexpr int NP = DE / 2;
  bool done = !active, conv = false;
  for (int sweep = 0;; ++sweep) {
    double off = 0.0;   // the convergence test in FP64 whatever T
    if (!done) {
      for (int idx = lt; idx < DE * DE; idx += W) {
        const int i = idx / DE, j = idx % DE;
        if (i != j) {
          const double x = (double)sar[i * LD + j];
          off = fma(x, x, off);
          if constexpr (CPLX) {
            const double y = (double)sai[i * LD + j];
            off = fma(y, y, off);
          }
        }
      }
    }
    off = seg_sum<W>(off);
    if (!done) {
      if (off <= tol2) { done = true; conv = true; }
      else if (sweep >= max_sweeps) { done = true; }
    }
    if (__all(done ? 1 : 0)) break;
    for (int r = 0; r < DE - 1; ++r) {
      if (!done) {
        for (int k = lt; k < NP; k += W) {
          int p, q;
          rr_pair(r, k, DE, p, q);
          const T xr = sar[p * LD + q];
          const T xi = CPLX ? sai[p * LD + q] : T(0);
          const T rr = CPLX ? dsqrt<T>(dfma<T>(xr, xr, xi * xi)) : fabs(xr);
          T t = T(0), cc = T(1), ss = T(0), er = T(1), ei = T(0);
          const T app = sar[p * LD + p], aqq = sar[q * LD + q];
          if (rr != T(0)) {
            rot_params<T>(app, aqq, rr, t, cc, ss);
            er = CPLX ? ddiv<T>(xr, rr) : copysign(T(1), xr);
            ei = CPLX ? ddiv<T>(-xi, rr) : T(0);
          }
          J.p[k] = p; J.q[k] = q;
          J.c[k] = cc; J.s[k] = ss; J.er[k] = er; J.ei[k] = ei;
          J.app[k] = app - t * rr;
          J.aqq[k] = aqq + t * rr;
        }
      }
      __syncthreads();
      if (!done) {
        // columns: A <- A G, U <- U G  (w = x_q e^{-i phi})
        for (int idx = lt; idx < DE * NP; idx += W) {
          const int i = idx % DE, k = idx / DE;
          const int p = J.p[k], q = J.q[k];
          const T cc = J.c[k], ss = J.s[k], er = J.er[k], ei = J.ei[k];
          {
            T pr = sar[i * LD + p], qr = sar[i * LD + q];
            T pi = CPLX ? sai[i * LD + p] : T(0), qi = CPLX ? sai[i * LD + q] : T(0);
            T wr = CPLX ? qr * er - qi * ei : qr * er;
            T wi = CPLX ? qr * ei + qi * er : T(0);
            sar[i * LD + p] = cc * pr - ss * wr;
            sar[i * LD + q] = ss * pr + cc * wr;
            if constexpr (CPLX) {
              sai[i * LD + p] = cc * pi - ss * wi;
              sai[i * LD + q] = ss * pi + cc * wi;
            }
          }
          if constexpr (VEC) {
            T pr = sur[i * LD + p], qr = sur[i * LD + q];
            T pi = CPLX ? sui[i * LD + p] : T(0), qi = CPLX ? sui[i * LD + q] : T(0);
            T wr = CPLX ? qr * er - qi * ei : qr * er;
            T wi = CPLX ? qr * ei + qi * er : T(0);
            sur[i * LD + p] = cc * pr - ss * wr;
            sur[i * LD + q] = ss * pr + cc * wr;
            if constexpr (CPLX) {
              sui[i * LD + p] = cc * pi - ss * wi;
              sui[i * LD + q] = ss * pi + cc * wi;
            }
          }
        }
      }
      __syncthreads();
      if (!done) {
        // rows: A <- G^H A  (w = x_q e^{+i phi})
        for (int idx = lt; idx < DE * NP; idx += W) {
          const int j = idx % DE, k = idx / DE;
          const int p = J.p[k], q = J.q[k];
          const T cc = J.c[k], ss = J.s[k], er = J.er[k], ei = -J.ei[k];
          T pr = sar[p * LD + j], qr = sar[q * LD + j];
          T pi = CPLX ? sai[p * LD + j] : T(0), qi = CPLX ? sai[q * LD + j] : T(0);
          T wr = CPLX ? qr * er - qi * ei : qr * er;
          T wi = CPLX ? qr * ei + qi * er : T(0);
          sar[p * LD + j] = cc * pr - ss * wr;
          sar[q * LD + j] = ss * pr + cc * wr;
          if constexpr (CPLX) {
            sai[p * LD + j] = cc * pi - ss * wi;
            sai[q * LD + j] = ss * pi + cc * wi;
          }
        }
      }
      __syncthreads();
      if (!done) {
        for (int k = lt; k < NP; k += W) {
          const int p = J.p[k], q = J.q[k];
          sar[p * LD + p] = J.app[k];
          sar[q * LD + q] = J.aqq[k];
          sar[p * LD + q] = T(0);
          sar[q * LD + p] = T(0);
          if constexpr (CPLX) {
            sai[p * LD + p] = T(0); sai[q * LD + q] = T(0);
            sai[p * LD + q] = T(0); sai[q * LD + p] = T(0);
          }
        }
      }
      __syncthreads();
    }
  }
  return conv;
}

// component k of a packed D x D Hermitian -> (i, j, imaginary?)
__device__ __forceinline__ void decode_comp(int k, int D, int& i, int& j, bool& im) {
  im = false;
  i = 0;
  if (k >= D * (D + 1) / 2) { im = true; k -= D * (D + 1) / 2; }
  const int rowlen0 = im ? D - 1 : D;
  while (k >= rowlen0 - i) { k -= rowlen0 - i; ++i; }
  j = i + k + (im ? 1 : 0);
}

// Write a cluster matrix Y (LDS) to its consumers: own marginal slot (if it has parents),
// the per-cluster output buffer, and the partial traces onto every child.
template <typename T, bool CPLX, int DE, int W>
__device__ void lds_outputs(const ClusterArgs<T>& A, int64_t c, int lt, int32_t gid, const T* yr, const T* yi) {
  constexpr int LD = DE + 1;
  constexpr int NB = log2i(DE);
  const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
  constexpr int NCE = n_comps(DE, CPLX);
  for (int k = lt; k < NCE; k += W) {
    int i, j;
    bool im;
    decode_comp(k, DE, i, j, im);
    const T v = im ? yi[i * LD + j] : yr[i * LD + j];
    if (rs_self >= 0 && A.R) A.R[(int64_t)k * A.S + rs_self] = v;
    if (A.marg) A.marg[A.marg_off[gid] + k] = v;
  }
  const int Dc = A.Dc;
  if (A.Tout && Dc > 0) {
    const int NR = DE / Dc;
    const int NCC = CPLX ? Dc * Dc : Dc * (Dc + 1) / 2;
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int mask = A.chmask[(int64_t)s * A.n + c];
      for (int k = lt; k < NCC; k += W) {
        int a, b;
        bool im;
        decode_comp(k, Dc, a, b, im);
        T sum = T(0);
        for (int x = 0; x < NR; ++x) {
          const int i = pdep_rt(a, x, mask, NB), j = pdep_rt(b, x, mask, NB);
          sum += im ? yi[i * LD + j] : yr[i * LD + j];
        }
        A.Tout[(int64_t)k * A.Mc + m] = sum;
      }
    }
  }
}

// Marginal weights from the eigenvalues on the diagonal of sar: Gibbs p (returns F_beta) or the
// normalised ground-space indicator (returns lambda_min).  Weights go to sp[].
template <typename T, int DE, int MODE, int W>
__device__ T lds_weights(const T* sar, T* sp, T lmin, T beta, T tau, int lt, bool active) {
  constexpr int LD = DE + 1;
  T w = T(0);
  if (active) {
    if constexpr (MODE == MODE_GIBBS) {
      for (int k = lt; k < DE; k += W) { T v = dexp<T>(-beta * (sar[k * LD + k] - lmin)); sp[k] = v; w += v; }
    } else {
      for (int k = lt; k < DE; k += W) { T v = (sar[k * LD + k] <= lmin + tau) ? T(1) : T(0); sp[k] = v; w += v; }
    }
  }
  const T Z = seg_sum<W>(w);
  __syncthreads();
  if (active)
    for (int k = lt; k < DE; k += W) sp[k] = ddiv<T>(sp[k], Z);
  __syncthreads();
  if constexpr (MODE == MODE_GIBBS) return lmin - ddiv<T>(dlog<T>(Z), beta);
  else return lmin;
}

// (yr, yi) = U diag(sp) U^H
template <typename T, bool CPLX, int DE, int W>
__device__ void lds_rebuild(const T* sur, const T* sui, const T* sp, T* yr, T* yi, int lt) {
  constexpr int LD = DE + 1;
  for (int idx = lt; idx < DE * DE; idx += W) {
    const int i = idx / DE, j = idx % DE;
    T sr = T(0), si = T(0);
    for (int k = 0; k < DE; ++k) {
      const T a_r = sur[i * LD + k] * sp[k];
      const T a_i = CPLX ? sui[i * LD + k] * sp[k] : T(0);
      sr = dfma<T>(a_r, sur[j * LD + k], sr);
      if constexpr (CPLX) {
        sr = dfma<T>(a_i, sui[j * LD + k], sr);
        si = dfma<T>(a_i, sur[j * LD + k], si);
        si = dfma<T>(-a_r, sui[j * LD + k], si);
      }
    }
    yr[i * LD + j] = sr;
    if constexpr (CPLX) yi[i * LD + j] = (i == j) ? T(0) : si;
  }
}

// W lanes per cluster, 64/W clusters per single-wave block.
template <typename T, bool CPLX, int DE, int MODE, int W>
__global__ __launch_bounds__(64) void k_cluster_lds(ClusterArgs<T> A) {
  constexpr int LD = DE + 1;
  constexpr int G = 64 / W;
  constexpr int SZ = DE * LD;
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  __shared__ T sar_[G * SZ];
  __shared__ T sai_[CPLX ? G * SZ : 1];
  __shared__ T sur_[VEC ? G * SZ : 1];
  __shared__ T sui_[(VEC && CPLX) ? G * SZ : 1];
  __shared__ JacobiScratch<T, DE / 2> J_[G];
  __shared__ T sp_[G * DE];
  const int g = threadIdx.x / W, lt = threadIdx.x % W;
  const int64_t c = (int64_t)blockIdx.x * G + g;
  const bool active = c < A.n;
  T* sar = sar_ + g * SZ;
  T* sai = CPLX ? sai_ + g * SZ : sai_;
  T* sur = VEC ? sur_ + g * SZ : sur_;
  T* sui = (VEC && CPLX) ? sui_ + g * SZ : sui_;
  T* sp = sp_ + g * DE;
  const T th = A.tab ? (T)A.tab->theta_cur : (T)A.theta;
  const T beta = A.tab ? (T)A.tab->beta : (T)A.beta;
  // ---- a1/a2: assemble theta_e at eta ----
  T n2 = T(0);
  if (active) n2 = lds_assemble<T, CPLX, DE, W>(A, c, lt, A.nu_c, A.ze_c, A.nu_p, A.ze_p, th, true, T(1), sar, sai);
  const T nrm2 = seg_sum<W>(n2);
  if constexpr (VEC) {
    if (active) {
      for (int idx = lt; idx < DE * DE; idx += W) {
        const int i = idx / DE, j = idx % DE;
        sur[i * LD + j] = (i == j) ? T(1) : T(0);
        if constexpr (CPLX) sui[i * LD + j] = T(0);
      }
    }
  }
  __syncthreads();
  // ---- a3: parallel cyclic Jacobi ----
  const bool conv = lds_jacobi<T, CPLX, DE, VEC, W>(sar, sai, sur, sui, J_[g], A.tol * A.tol * (double)nrm2,
                                                    A.max_sweeps, lt, active);
  if (active && !conv && lt == 0 && A.noconv) atomicAdd(A.noconv, 1ull);
  T lmin = T(INFINITY);
  if (active)
    for (int k = lt; k < DE; k += W) lmin = fmin(lmin, sar[k * LD + k]);
  lmin = seg_min<W>(lmin);
  if (active && lt == 0 && !isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  const int32_t gid = active ? A.gid[c] : 0;
  if constexpr (MODE == MODE_CERTIFY) {
    // remaining off-diagonal mass (Weyl, as in the register kernel)
    double off2 = 0.0;
    if (active)
      for (int idx = lt; idx < DE * DE; idx += W) {
        const int i = idx / DE, j = idx % DE;
        if (i == j) continue;
        const double xr = (double)sar[i * LD + j];
        off2 = fma(xr, xr, off2);
        if constexpr (CPLX) {
          const double xi = (double)sai[i * LD + j];
          off2 = fma(xi, xi, off2);
        }
      }
    off2 = seg_sum<W>(off2);
    if (active && lt == 0) {
      A.scal[gid] = (double)lmin;
      A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt((double)nrm2) + sqrt(off2);
    }
  } else {
    // ---- a4: weights and the marginal U diag(p) U^H (over A) ----
    const T val = lds_weights<T, DE, MODE, W>(sar, sp, lmin, beta, (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2)), lt,
                                              active);
    if (active && lt == 0 && A.scal) A.scal[gid] = (double)val;
    if (active) lds_rebuild<T, CPLX, DE, W>(sur, sui, sp, sar, sai, lt);
    __syncthreads();
    // ---- a5: outputs ----
    if (active) lds_outputs<T, CPLX, DE, W>(A, c, lt, gid, sar, sai);
  }
}

// ------------------------------------------------------------------------------------------
// clusters holding a spin-1 site (De = 3, 9, 27, 6, ... <= 64): the LDS Jacobi kernel driven by
// index tables instead of site bit masks, the De x De problem embedded in DEP x DEP (DEP the next
// power of two) with decoupled padding
// ------------------------------------------------------------------------------------------
//
// The padding indices De..DEP-1 carry a diagonal above every eigenvalue of theta_e and zero
// off-diagonal entries.  A Jacobi rotation of a pair with a zero off-diagonal is the identity
// (c = 1, s = 0) and a rotation of two other indices keeps zeros zero, so the padding indices stay
// eigenvectors e_k with their own diagonal: they are left out of lambda_min, the weights, the norms
// and the outputs by index.

template <typename T, bool CPLX, int DEP, int W>
__device__ T gen_assemble(const ClusterArgs<T>& A, int64_t c, int lt, T th, T* dr, T* di) {
  constexpr int LD = DEP + 1;
  const int De = A.De, Dc = A.Dc;
  const int64_t ho = A.hoff[c];
  T my_n2 = T(0);
  for (int idx = lt; idx < DEP * DEP; idx += W) {
    const int i = idx / DEP, j = idx % DEP;
    T vr = T(0), vi = T(0);
    if (i < De && j < De) {
      if (ho >= 0) herm_elem<T>([&](int k) { return (T)A.h[ho + k]; }, i, j, De, CPLX, vr, vi);
      for (int s = 0; s < A.maxch; ++s) {
        const int m = A.ch[(int64_t)s * A.n + c];
        if (m < 0) continue;
        const int32_t* g = A.gtab + ((int64_t)s * A.n + c) * De;
        const int ei = g[i], ej = g[j];
        if (((ei >> 8) & 0xff) != ((ej >> 8) & 0xff)) continue;   // different remaining index
        const int a = ei & 0xff, b = ej & 0xff;
        T er, eim;
        if (A.ze_c)
          herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mc + m;
                                    return extrap<T>(A.nu_c[o], A.ze_c[o], th); }, a, b, Dc, CPLX, er, eim);
        else
          herm_elem<T>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, a, b, Dc, CPLX, er, eim);
        vr -= er;
        vi -= eim;
      }
      for (int s = 0; s < A.maxpar; ++s) {
        const int m = A.par[(int64_t)s * A.n + c];
        if (m < 0) continue;
        T er, eim;
        if (A.ze_p)
          herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mp + m;
                                    return extrap<T>(A.nu_p[o], A.ze_p[o], th); }, i, j, De, CPLX, er, eim);
        else
          herm_elem<T>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, i, j, De, CPLX, er, eim);
        vr += er;
        vi += eim;
      }
      my_n2 = dfma<T>(vr, vr, my_n2);
      if constexpr (CPLX) my_n2 = dfma<T>(vi, vi, my_n2);
    }
    dr[i * LD + j] = vr;
    if constexpr (CPLX) di[i * LD + j] = vi;
  }
  return my_n2;
}

template <typename T, bool CPLX, int DEP, int W>
__device__ void gen_outputs(const ClusterArgs<T>& A, int64_t c, int lt, int32_t gid, const T* yr, const T* yi) {
  constexpr int LD = DEP + 1;
  const int De = A.De, Dc = A.Dc;
  const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
  const int NCE = CPLX ? De * De : De * (De + 1) / 2;
  for (int k = lt; k < NCE; k += W) {
    int i, j;
    bool im;
    decode_comp(k, De, i, j, im);
    const T v = im ? yi[i * LD + j] : yr[i * LD + j];
    if (rs_self >= 0 && A.R) A.R[(int64_t)k * A.S + rs_self] = v;
    if (A.marg) A.marg[A.marg_off[gid] + k] = v;
  }
  if (A.Tout && Dc > 0) {
    const int NR = De / Dc;
    const int NCC = CPLX ? Dc * Dc : Dc * (Dc + 1) / 2;
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int32_t* g = A.gtab + ((int64_t)s * A.n + c) * De;
      for (int k = lt; k < NCC; k += W) {
        int a, b;
        bool im;
        decode_comp(k, Dc, a, b, im);
        T sum = T(0);
        for (int x = 0; x < NR; ++x) {
          const int i = g[a * NR + x] >> 16, j = g[b * NR + x] >> 16;
          sum += im ? yi[i * LD + j] : yr[i * LD + j];
        }
        A.Tout[(int64_t)k * A.Mc + m] = sum;
      }
    }
  }
}

template <typename T, bool CPLX, int DEP, int MODE, int W>
__global__ __launch_bounds__(64) void k_cluster_gen(ClusterArgs<T> A) {
  constexpr int LD = DEP + 1;
  constexpr int G = 64 / W;
  constexpr int SZ = DEP * LD;
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  __shared__ T sar_[G * SZ];
  __shared__ T sai_[CPLX ? G * SZ : 1];
  __shared__ T sur_[VEC ? G * SZ : 1];
  __shared__ T sui_[(VEC && CPLX) ? G * SZ : 1];
  __shared__ JacobiScratch<T, DEP / 2> J_[G];
  __shared__ T sp_[G * DEP];
  const int g = threadIdx.x / W, lt = threadIdx.x % W;
  const int64_t c = (int64_t)blockIdx.x * G + g;
  const bool active = c < A.n;
  const int De = A.De;
  T* sar = sar_ + g * SZ;
  T* sai = CPLX ? sai_ + g * SZ : sai_;
  T* sur = VEC ? sur_ + g * SZ : sur_;
  T* sui = (VEC && CPLX) ? sui_ + g * SZ : sui_;
  T* sp = sp_ + g * DEP;
  const T th = A.tab ? (T)A.tab->theta_cur : (T)A.theta;
  const T beta = A.tab ? (T)A.tab->beta : (T)A.beta;
  // ---- a1/a2: assemble theta_e at eta, then the padding diagonal ----
  T n2 = T(0);
  if (active) n2 = gen_assemble<T, CPLX, DEP, W>(A, c, lt, th, sar, sai);
  const T nrm2 = seg_sum<W>(n2);
  __syncthreads();
  if (active)
    for (int k = De + lt; k < DEP; k += W) sar[k * LD + k] = T(2) * dsqrt<T>(nrm2) + T(1);   // > every eigenvalue
  if constexpr (VEC) {
    if (active) {
      for (int idx = lt; idx < DEP * DEP; idx += W) {
        const int i = idx / DEP, j = idx % DEP;
        sur[i * LD + j] = (i == j) ? T(1) : T(0);
        if constexpr (CPLX) sui[i * LD + j] = T(0);
      }
    }
  }
  __syncthreads();
  // ---- a3: parallel cyclic Jacobi over DEP (the padding stays decoupled) ----
  const bool conv = lds_jacobi<T, CPLX, DEP, VEC, W>(sar, sai, sur, sui, J_[g], A.tol * A.tol * (double)nrm2,
                                                     A.max_sweeps, lt, active);
  if (active && !conv && lt == 0 && A.noconv) atomicAdd(A.noconv, 1ull);
  T lmin = T(INFINITY);
  if (active)
    for (int k = lt; k < De; k += W) lmin = fmin(lmin, sar[k * LD + k]);
  lmin = seg_min<W>(lmin);
  if (active && lt == 0 && !isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  const int32_t gid = active ? A.gid[c] : 0;
  if constexpr (MODE == MODE_CERTIFY) {
    double off2 = 0.0;   // off-diagonal mass left by the sweeps (Weyl)
    if (active)
      for (int idx = lt; idx < DEP * DEP; idx += W) {
        const int i = idx / DEP, j = idx % DEP;
        if (i == j) continue;
        const double xr = (double)sar[i * LD + j];
        off2 = fma(xr, xr, off2);
        if constexpr (CPLX) {
          const double xi = (double)sai[i * LD + j];
          off2 = fma(xi, xi, off2);
        }
      }
    off2 = seg_sum<W>(off2);
    if (active && lt == 0) {
      A.scal[gid] = (double)lmin;
      A.scal2[gid] = 8.0 * De * DBL_EPSILON * sqrt((double)nrm2) + sqrt(off2);
    }
  } else {
    // ---- a4: weights (padding indices excluded) and the marginal U diag(p) U^H ----
    T w = T(0);
    if (active) {
      const T tau = (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2));
      for (int k = lt; k < DEP; k += W) {
        T v = T(0);
        if (k < De) {
          if constexpr (MODE == MODE_GIBBS) v = dexp<T>(-beta * (sar[k * LD + k] - lmin));
          else v = (sar[k * LD + k] <= lmin + tau) ? T(1) : T(0);
        }
        sp[k] = v;
        w += v;
      }
    }
    const T Z = seg_sum<W>(w);
    __syncthreads();
    if (active)
      for (int k = lt; k < DEP; k += W) sp[k] = ddiv<T>(sp[k], Z);
    __syncthreads();
    const T val = (MODE == MODE_GIBBS) ? lmin - ddiv<T>(dlog<T>(Z), beta) : lmin;
    if (active && lt == 0 && A.scal) A.scal[gid] = (double)val;
    if (active) lds_rebuild<T, CPLX, DEP, W>(sur, sui, sp, sar, sai, lt);
    __syncthreads();
    // ---- a5: outputs ----
    if (active) gen_outputs<T, CPLX, DEP, W>(A, c, lt, gid, sar, sai);
  }
}

// ------------------------------------------------------------------------------------------
// large clusters (De = 128, 256): one 1024-thread workgroup per cluster
// ------------------------------------------------------------------------------------------
//
// A De x De complex matrix and its eigenvectors do not fit one CU's LDS, so theta_e, U and
// rho live in a per-workgroup scratch slab in HBM (the workgroup walks clusters with a grid
// stride); the round-robin parallel Jacobi applies De/2 disjoint rotations per round with all
// 1024 threads.  The reconstruction rho = W W^H with W = U diag(sqrt p) is a dense contraction
// and runs on the matrix cores: v_mfma_f32_32x32x2_f32 (FP32) / v_mfma_f64_16x16x4_f64 (FP64),
// four real products per complex tile.

typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = T(0);
  const int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}
template <typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
  const int nw = blockDim.x / 64;
  for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
  __syncthreads();
  return s;
}
template <typename T>
__device__ __forceinline__ T block_min(T v, T* red) {
  v = wave_min(v);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
  const int nw = blockDim.x / 64;
  for (int i = 1; i < nw; ++i) s = fmin(s, red[i]);
  __syncthreads();
  return s;
}

// rho tile accumulation on the matrix cores; (wr, wi) = W rows, rho written to (orr, ori)
template <typename T, bool CPLX>
__device__ void mfma_rebuild(const T* ur, const T* ui, const T* sq, T* orr, T* ori, int D) {
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64, nw = blockDim.x / 64;
  if constexpr (std::is_same<T, float>::value) {
    const int nt = D / 32;
    for (int tile = wave; tile < nt * nt; tile += nw) {
      const int I = tile / nt, J = tile % nt;
      mfma_f32x16 cr = {0}, ci = {0};
      const int i = I * 32 + (l % 32), j = J * 32 + (l % 32);
      for (int k0 = 0; k0 < D; k0 += 2) {
        const int k = k0 + l / 32;
        const float s = sq[k];
        const float ar = ur[(int64_t)i * D + k] * s, br = ur[(int64_t)j * D + k] * s;
        cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, cr, 0, 0, 0);
        if constexpr (CPLX) {
          const float ai = ui[(int64_t)i * D + k] * s, bi = ui[(int64_t)j * D + k] * s;
          cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar, bi, ci, 0, 0, 0);
        }
      }
      for (int r = 0; r < 16; ++r) {
        const int row = I * 32 + 8 * (r / 4) + 4 * (l / 32) + (r % 4), col = J * 32 + (l % 32);
        orr[(int64_t)row * D + col] = cr[r];
        if constexpr (CPLX) ori[(int64_t)row * D + col] = (row == col) ? 0.f : ci[r];
      }
    }
  } else {
    const int nt = D / 16;
    for (int tile = wave; tile < nt * nt; tile += nw) {
      const int I = tile / nt, J = tile % nt;
      mfma_f64x4 cr = {0}, ci = {0};
      const int i = I * 16 + (l % 16), j = J * 16 + (l % 16);
      for (int k0 = 0; k0 < D; k0 += 4) {
        const int k = k0 + l / 16;
        const double s = sq[k];
        const double ar = ur[(int64_t)i * D + k] * s, br = ur[(int64_t)j * D + k] * s;
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cr, 0, 0, 0);
        if constexpr (CPLX) {
          const double ai = ui[(int64_t)i * D + k] * s, bi = ui[(int64_t)j * D + k] * s;
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar, bi, ci, 0, 0, 0);
        }
      }
      for (int r = 0; r < 4; ++r) {
        const int row = I * 16 + 4 * r + (l / 16), col = J * 16 + (l % 16);
        orr[(int64_t)row * D + col] = cr[r];
        if constexpr (CPLX) ori[(int64_t)row * D + col] = (row == col) ? 0.0 : ci[r];
      }
    }
  }
}

// theta_e of cluster c assembled element by element into a row-major D x D slab (ar, ai) of
// element type S; with VEC the slab (ur, ui) is set to the identity.  Returns this thread's
// share of ||theta||_F^2.
// Element (i, j) of theta_e for cluster c: h_e, minus the lifted child messages, plus the parent
// messages (extrapolated with weight th when the zeta pointers are set).
template <typename T, bool CPLX>
__device__ __forceinline__ void theta_elem(const ClusterArgs<T>& A, int64_t c, int D, int NB, int64_t ho, int i, int j,
                                           T th, T& vr, T& vi) {
  const int Dc = A.Dc;
  vr = T(0);
  vi = T(0);
  if (ho >= 0) herm_elem<T>([&](int k) { return (T)A.h[ho + k]; }, i, j, D, CPLX, vr, vi);
  for (int s = 0; s < A.maxch; ++s) {
    const int m = A.ch[(int64_t)s * A.n + c];
    if (m < 0) continue;
    const int mask = A.chmask[(int64_t)s * A.n + c];
    if (((i ^ j) & ~mask & (D - 1)) != 0) continue;
    const int a = pext_rt(i, mask, NB), b = pext_rt(j, mask, NB);
    T er, ei;
    if (A.ze_c)
      herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mc + m;
                                return extrap<T>(A.nu_c[o], A.ze_c[o], th); }, a, b, Dc, CPLX, er, ei);
    else
      herm_elem<T>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, a, b, Dc, CPLX, er, ei);
    vr -= er;
    vi -= ei;
  }
  for (int s = 0; s < A.maxpar; ++s) {
    const int m = A.par[(int64_t)s * A.n + c];
    if (m < 0) continue;
    T er, ei;
    if (A.ze_p)
      herm_elem<T>([&](int k) { const int64_t o = (int64_t)k * A.Mp + m;
                                return extrap<T>(A.nu_p[o], A.ze_p[o], th); }, i, j, D, CPLX, er, ei);
    else
      herm_elem<T>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, i, j, D, CPLX, er, ei);
    vr += er;
    vi += ei;
  }
}

template <typename T, typename S, bool CPLX, bool VEC>
__device__ T big_assemble(const ClusterArgs<T>& A, int64_t c, int D, S* ar, S* ai, S* ur, S* ui, T th, int tid,
                          int nth) {
  const int NB = log2i(D);
  const int64_t DD = (int64_t)D * D;
  const int64_t ho = A.hoff[c];
  T my_n2 = T(0);
  for (int64_t idx = tid; idx < DD; idx += nth) {
    const int i = (int)(idx / D), j = (int)(idx % D);
    T vr, vi;
    theta_elem<T, CPLX>(A, c, D, NB, ho, i, j, th, vr, vi);
    ar[idx] = (S)vr;
    if constexpr (CPLX) ai[idx] = (S)vi;
    if constexpr (VEC) {
      ur[idx] = (i == j) ? S(1) : S(0);
      if constexpr (CPLX) ui[idx] = S(0);
    }
    my_n2 = dfma<T>(vr, vr, my_n2);
    if constexpr (CPLX) my_n2 = dfma<T>(vi, vi, my_n2);
  }
  return my_n2;
}

// Outputs of a cluster whose marginal scale * (rr, ri) sits in a row-major slab: own marginal
// slot, per-cluster marginal, partial traces onto every child.
template <typename T, typename S, bool CPLX>
__device__ void big_outputs(const ClusterArgs<T>& A, int64_t c, int D, int32_t gid, const S* rr_, const S* ri_,
                            S scale, int tid, int nth) {
  const int NB = log2i(D);
  const int Dc = A.Dc;
  const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
  const int NCE = CPLX ? D * D : D * (D + 1) / 2;
  for (int k = tid; k < NCE; k += nth) {
    int i, j;
    bool im;
    decode_comp(k, D, i, j, im);
    const T v = (T)(scale * (im ? ri_[(int64_t)i * D + j] : rr_[(int64_t)i * D + j]));
    if (rs_self >= 0 && A.R) A.R[(int64_t)k * A.S + rs_self] = v;
    if (A.marg) A.marg[A.marg_off[gid] + k] = v;
  }
  if (A.Tout && Dc > 0) {
    const int NR = D / Dc;
    const int NCC = CPLX ? Dc * Dc : Dc * (Dc + 1) / 2;
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int mask = A.chmask[(int64_t)s * A.n + c];
      for (int k = tid; k < NCC; k += nth) {
        int a, b;
        bool im;
        decode_comp(k, Dc, a, b, im);
        S sum = S(0);
        for (int x = 0; x < NR; ++x) {
          const int i = pdep_rt(a, x, mask, NB), j = pdep_rt(b, x, mask, NB);
          sum += im ? ri_[(int64_t)i * D + j] : rr_[(int64_t)i * D + j];
        }
        A.Tout[(int64_t)k * A.Mc + m] = (T)(scale * sum);
      }
    }
  }
}

template <typename T, bool CPLX, int MODE>
__global__ __launch_bounds__(1024) void k_cluster_big(ClusterArgs<T> A, T* scratch, int64_t slab) {
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  __shared__ T cs_c[128], cs_s[128], cs_er[128], cs_ei[128], cs_app[128], cs_aqq[128];
  __shared__ int cs_p[128], cs_q[128];
  __shared__ T red[16];
  __shared__ double redd[16];
  __shared__ T sp[256];
  const int D = A.De;
  const int NB = log2i(D);
  const int NP = D / 2;
  const int64_t DD = (int64_t)D * D;
  T* ar = scratch + (int64_t)blockIdx.x * slab;
  T* ai = ar + DD;   // unused for real problems
  T* ur = ar + (CPLX ? 2 : 1) * DD;
  T* ui = ur + DD;
  T* rr_ = ar + (CPLX ? 4 : 2) * DD;
  T* ri_ = rr_ + DD;
  const int tid = threadIdx.x, nth = blockDim.x;
  const T th = A.tab ? (T)A.tab->theta_cur : (T)A.theta;
  const T beta = A.tab ? (T)A.tab->beta : (T)A.beta;
  for (int64_t c = blockIdx.x; c < A.n; c += gridDim.x) {
    // ---- a2: assemble theta_e ----
    const int Dc = A.Dc;
    const T my_n2 = big_assemble<T, T, CPLX, VEC>(A, c, D, ar, ai, ur, ui, th, tid, nth);
    const T nrm2 = block_sum(my_n2, red);
    // ---- a3: parallel cyclic Jacobi over the slab ----
    const double tol2 = A.tol * A.tol * (double)nrm2;
    bool conv = false;
    for (int sweep = 0; sweep <= A.max_sweeps; ++sweep) {
      double off = 0.0;   // the convergence test in FP64 whatever T
      for (int64_t idx = tid; idx < DD; idx += nth) {
        if (idx / D != idx % D) {
          const double x = (double)ar[idx];
          off = fma(x, x, off);
          if constexpr (CPLX) {
            const double y = (double)ai[idx];
            off = fma(y, y, off);
          }
        }
      }
      off = block_sum(off, redd);
      if (off <= tol2) { conv = true; break; }
      if (sweep == A.max_sweeps) break;
      for (int r = 0; r < D - 1; ++r) {
        if (tid < NP) {
          int p, q;
          rr_pair(r, tid, D, p, q);
          const T xr = ar[(int64_t)p * D + q];
          const T xi = CPLX ? ai[(int64_t)p * D + q] : T(0);
          const T rr = CPLX ? dsqrt<T>(dfma<T>(xr, xr, xi * xi)) : fabs(xr);
          T t = T(0), cc = T(1), ss = T(0), er = T(1), ei = T(0);
          const T app = ar[(int64_t)p * D + p], aqq = ar[(int64_t)q * D + q];
          if (rr != T(0)) {
            rot_params<T>(app, aqq, rr, t, cc, ss);
            er = CPLX ? ddiv<T>(xr, rr) : copysign(T(1), xr);
            ei = CPLX ? ddiv<T>(-xi, rr) : T(0);
          }
          cs_p[tid] = p; cs_q[tid] = q;
          cs_c[tid] = cc; cs_s[tid] = ss; cs_er[tid] = er; cs_ei[tid] = ei;
          cs_app[tid] = app - t * rr;
          cs_aqq[tid] = aqq + t * rr;
        }
        __syncthreads();
        for (int idx = tid; idx < D * NP; idx += nth) {
          const int i = idx % D, k = idx / D;
          const int p = cs_p[k], q = cs_q[k];
          const T cc = cs_c[k], ss = cs_s[k], er = cs_er[k], ei = cs_ei[k];
          {
            const int64_t op = (int64_t)i * D + p, oq = (int64_t)i * D + q;
            T pr = ar[op], qr = ar[oq];
            T pi = CPLX ? ai[op] : T(0), qi = CPLX ? ai[oq] : T(0);
            T wr = CPLX ? qr * er - qi * ei : qr * er;
            T wi = CPLX ? qr * ei + qi * er : T(0);
            ar[op] = cc * pr - ss * wr;
            ar[oq] = ss * pr + cc * wr;
            if constexpr (CPLX) { ai[op] = cc * pi - ss * wi; ai[oq] = ss * pi + cc * wi; }
          }
          if constexpr (VEC) {
            const int64_t op = (int64_t)i * D + p, oq = (int64_t)i * D + q;
            T pr = ur[op], qr = ur[oq];
            T pi = CPLX ? ui[op] : T(0), qi = CPLX ? ui[oq] : T(0);
            T wr = CPLX ? qr * er - qi * ei : qr * er;
            T wi = CPLX ? qr * ei + qi * er : T(0);
            ur[op] = cc * pr - ss * wr;
            ur[oq] = ss * pr + cc * wr;
            if constexpr (CPLX) { ui[op] = cc * pi - ss * wi; ui[oq] = ss * pi + cc * wi; }
          }
        }
        __syncthreads();
        for (int idx = tid; idx < D * NP; idx += nth) {
          const int j = idx % D, k = idx / D;
          const int p = cs_p[k], q = cs_q[k];
          const T cc = cs_c[k], ss = cs_s[k], er = cs_er[k], ei = -cs_ei[k];
          const int64_t op = (int64_t)p * D + j, oq = (int64_t)q * D + j;
          T pr = ar[op], qr = ar[oq];
          T pi = CPLX ? ai[op] : T(0), qi = CPLX ? ai[oq] : T(0);
          T wr = CPLX ? qr * er - qi * ei : qr * er;
          T wi = CPLX ? qr * ei + qi * er : T(0);
          ar[op] = cc * pr - ss * wr;
          ar[oq] = ss * pr + cc * wr;
          if constexpr (CPLX) { ai[op] = cc * pi - ss * wi; ai[oq] = ss * pi + cc * wi; }
        }
        __syncthreads();
        if (tid < NP) {
          const int p = cs_p[tid], q = cs_q[tid];
          ar[(int64_t)p * D + p] = cs_app[tid];
          ar[(int64_t)q * D + q] = cs_aqq[tid];
          ar[(int64_t)p * D + q] = T(0);
          ar[(int64_t)q * D + p] = T(0);
          if constexpr (CPLX) {
            ai[(int64_t)p * D + p] = T(0); ai[(int64_t)q * D + q] = T(0);
            ai[(int64_t)p * D + q] = T(0); ai[(int64_t)q * D + p] = T(0);
          }
        }
        __syncthreads();
      }
    }
    if (!conv && tid == 0 && A.noconv) atomicAdd(A.noconv, 1ull);
    T lmin = T(INFINITY);
    for (int k = tid; k < D; k += nth) lmin = fmin(lmin, ar[(int64_t)k * D + k]);
    lmin = block_min(lmin, red);
    if (tid == 0 && !isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
    const int32_t gid = A.gid[c];
    if constexpr (MODE == MODE_CERTIFY) {
      if (tid == 0) {
        A.scal[gid] = (double)lmin;
        A.scal2[gid] = 8.0 * D * DBL_EPSILON * sqrt((double)nrm2);
      }
    } else {
      // ---- a4: weights (sqrt stored for the W W^H product) ----
      T w = T(0);
      for (int k = tid; k < D; k += nth) {
        const T lk = ar[(int64_t)k * D + k];
        T v;
        if constexpr (MODE == MODE_GIBBS) v = dexp<T>(-beta * (lk - lmin));
        else v = (lk <= lmin + (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2))) ? T(1) : T(0);
        sp[k] = v;
        w += v;
      }
      const T Z = block_sum(w, red);
      for (int k = tid; k < D; k += nth) sp[k] = dsqrt<T>(sp[k] / Z);
      if (tid == 0 && A.scal) A.scal[gid] = (MODE == MODE_GIBBS) ? (double)(lmin - dlog<T>(Z) / beta) : (double)lmin;
      __syncthreads();
      mfma_rebuild<T, CPLX>(ur, ui, sp, rr_, ri_, D);
      __syncthreads();
      // ---- a5: outputs ----
      big_outputs<T, T, CPLX>(A, c, D, gid, rr_, ri_, T(1), tid, nth);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Gibbs state by scaling and squaring on the matrix cores (accelerated iteration, De = 16, 32)
// ------------------------------------------------------------------------------------------
//
// The smoothed dual needs rho_e = exp(-beta theta_e) / Z and F_beta = -(1/beta) log Z only
// (Sec. 4.1.2); the eigenvectors are not needed for that.  With mu = Tr(theta)/D and
// X = beta (theta - mu), the scaling s is the least s >= 0 with ||X|| / 2^s <= 1/2, where ||X||
// is an upper bound of the spectral norm: the induced 1-norm (largest absolute row sum) in the
// one-wave kernel, min(||X||_F, ||X||_1) in the workgroup kernel (both norms are
// submultiplicative, so the Taylor remainder bound holds in either; the 1-norm is the tight one
// for lifted local terms 1 (x) h, whose Frobenius norm carries a factor sqrt(D / D_h)), and
//     E0 = T_m(-X / 2^s)                (Taylor polynomial, Paterson-Stockmeyer, p = 3; m = 12,
//                                        or 8 for float messages)
//     Y0 = E0 / tau_0,  Y_j = Y_{j-1}^2 / tau_j    (j = 1..s)
//     rho = Y_s / Tr Y_s,  log Z = 2^s log tau_0 + sum_j 2^(s-j) log tau_j + log Tr Y_s
// for any positive rescalings tau_j (the one-wave kernel uses exact powers of two; the
// workgroup kernel tau_0 = Tr E0, tau_j = (Tr Y_{j-1})^2).
// The truncation error of T12 at norm 1/2 is below 2e-14 relative (in the norm that set s),
// i.e. a backward error of about 7e-14 ||X|| in X, which exact squaring preserves (T8: 5.4e-9,
// under the float rounding of the messages).  Rounding in the squarings adds a relative error of
// order D u (spectral spread / gap) to rho: the part along the dominant eigenvector is removed
// by the final trace normalisation, the rest is damped once the spectrum separates.  The
// polynomial and the first four squarings run in FP64 on the matrix cores; with double messages
// so do the rest, with float messages the later squarings run in FP32.
//
// One wavefront per cluster.  A matrix is NB x NB blocks of 16 x 16 held in the MFMA result
// layout: lane l, register r of block (I, J) is element (16 I + 4 r + l/16, 16 J + l%16).
// Every matrix here is Hermitian (a polynomial in X), so the A operand of block (I, K) at
// k-step kk, element (16 I + l%16, 16 K + 4 kk + l/16), is the conjugate of register kk of
// block (K, I): both operands come straight from the registers, with no data movement.
constexpr int kExpmLut = 8;   // children handled through the LDS index tables (more: generic path)
constexpr int kF64Squarings = 4;   // float-message path: squarings kept in FP64 before the FP32 ones

// pext and pdep over the site bits of a one-wave cluster (at most 5 sites), for every site mask,
// built at compile time: pext[mask][i] packs the bits of i at the mask positions;
// pdepN[mask][(a << lnr) | x] places the bits of a at the mask positions and those of x at the
// other N - popcount(mask) = lnr positions.
struct SiteBitTables {
  unsigned char pext[32][32];
  unsigned char pdep4[16][16];
  unsigned char pdep5[32][32];
};
constexpr SiteBitTables make_site_bit_tables() {
  SiteBitTables t{};
  for (int m = 0; m < 32; ++m)
    for (int i = 0; i < 32; ++i) t.pext[m][i] = (unsigned char)pext_bits(i, m, 5);
  for (int m = 0; m < 16; ++m) {
    const int lnr = 4 - __builtin_popcount(m);
    for (int p = 0; p < 16; ++p) t.pdep4[m][p] = (unsigned char)pdep_bits(p >> lnr, p & ((1 << lnr) - 1), m, 4);
  }
  for (int m = 0; m < 32; ++m) {
    const int lnr = 5 - __builtin_popcount(m);
    for (int p = 0; p < 32; ++p) t.pdep5[m][p] = (unsigned char)pdep_bits(p >> lnr, p & ((1 << lnr) - 1), m, 5);
  }
  return t;
}
static __constant__ SiteBitTables kSiteBits = make_site_bit_tables();

template <int NB, bool CPLX>
struct XMat {
  double re[NB][NB][4];
  double im[CPLX ? NB : 1][CPLX ? NB : 1][4];
};

// C (+)= X Y for Hermitian X; C accumulates onto its contents, column block by column block,
// so C may alias Y (never X).
template <int NB, bool CPLX>
__device__ __forceinline__ void xmm(const XMat<NB, CPLX>& X, const XMat<NB, CPLX>& Y, XMat<NB, CPLX>& C) {
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    mfma_f64x4 cr[NB], ci[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[I][r] = C.re[I][J][r];
        if constexpr (CPLX) ci[I][r] = C.im[I][J][r];
      }
#pragma unroll
      for (int K = 0; K < NB; ++K)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          cr[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(X.re[K][I][kk], Y.re[K][J][kk], cr[I], 0, 0, 0);
          if constexpr (CPLX) {
            cr[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(X.im[K][I][kk], Y.im[K][J][kk], cr[I], 0, 0, 0);
            ci[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(X.re[K][I][kk], Y.im[K][J][kk], ci[I], 0, 0, 0);
            ci[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(-X.im[K][I][kk], Y.re[K][J][kk], ci[I], 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C.re[I][J][r] = cr[I][r];
        if constexpr (CPLX) C.im[I][J][r] = ci[I][r];
      }
  }
}

// lane-local diagonal test for register r of a diagonal block
__device__ __forceinline__ bool xdiag(int r, int l) { return 4 * r + (l >> 4) == (l & 15); }

// FP32 matrices for the last squarings of the float-message path, in the v_mfma_f32_16x16x4_f32
// result layout: lane l, register r of block (I, J) is element (16 I + 4 (l/16) + r, 16 J + l%16).
// Lane group g = l/16 supplies the k index 4 g + kk at k-step kk, so for Hermitian X the A operand
// of block (I, K) is the conjugate of register kk of block (K, I), as in the FP64 layout.
template <int NB, bool CPLX>
struct XMat32 {
  float re[NB][NB][4];
  float im[CPLX ? NB : 1][CPLX ? NB : 1][4];
};
typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));

template <int NB, bool CPLX>
__device__ __forceinline__ void xmm32(const XMat32<NB, CPLX>& X, const XMat32<NB, CPLX>& Y, XMat32<NB, CPLX>& C) {
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    mfma_f32x4 cr[NB], ci[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[I][r] = C.re[I][J][r];
        if constexpr (CPLX) ci[I][r] = C.im[I][J][r];
      }
#pragma unroll
      for (int K = 0; K < NB; ++K)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          cr[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(X.re[K][I][kk], Y.re[K][J][kk], cr[I], 0, 0, 0);
          if constexpr (CPLX) {
            cr[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(X.im[K][I][kk], Y.im[K][J][kk], cr[I], 0, 0, 0);
            ci[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(X.re[K][I][kk], Y.im[K][J][kk], ci[I], 0, 0, 0);
            ci[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(-X.im[K][I][kk], Y.re[K][J][kk], ci[I], 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C.re[I][J][r] = cr[I][r];
        if constexpr (CPLX) C.im[I][J][r] = ci[I][r];
      }
  }
}

// Trace of an FP32-layout matrix: the diagonal sits in lanes whose 4-lane group (l % 16) / 4
// equals l / 16 (lanes 0-3, 20-23, 40-43, 60-63), register l % 4; two quad-permute DPP steps
// and four readlanes sum it.  Used only for the binary exponent of the rescaling steps.
template <int CTRL>
__device__ __forceinline__ float dpp_movf(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int NB, bool CPLX>
__device__ __forceinline__ float xtrace32(const XMat32<NB, CPLX>& M, int l) {
  float v = 0.f;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * (l >> 4) + r == (l & 15)) v += M.re[I][I][r];
  v += dpp_movf<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_movf<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  const auto rl = [&](int lane) { return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane)); };
  return (rl(0) + rl(20)) + (rl(40) + rl(60));
}

template <int NB, bool CPLX>
__device__ __forceinline__ void xzero(XMat<NB, CPLX>& M) {
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        M.re[I][J][r] = 0.0;
        if constexpr (CPLX) M.im[I][J][r] = 0.0;
      }
}

// Trace of an FP64-layout matrix: the diagonal sits in lanes with l % 4 == l / 16, register
// (l % 16) / 4 of every diagonal block, four lanes 4 apart in each row of 16.  Two row-shift
// DPP steps leave each row's sum in its lane 12 + l / 16; four readlanes add the rows.
template <int NB, bool CPLX>
__device__ __forceinline__ double xtrace(const XMat<NB, CPLX>& M, int l) {
  double v = 0.0;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (xdiag(r, l)) v += M.re[I][I][r];
  v += dpp_mov<0x114>(v);   // row_shr:4
  v += dpp_mov<0x118>(v);   // row_shr:8
  return (readlane_d(v, 12) + readlane_d(v, 29)) + (readlane_d(v, 46) + readlane_d(v, 63));
}

// FP32 estimate of the trace of an FP64-layout matrix, for the binary exponent of a rescaling
// (the value only picks an exact power of two): the diagonal lanes as in xtrace, the sum in FP32.
template <int NB, bool CPLX>
__device__ __forceinline__ float xtrace_est(const XMat<NB, CPLX>& M, int l) {
  double t = 0.0;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (xdiag(r, l)) t += M.re[I][I][r];
  float v = (float)t;
  v += dpp_movf<0x114>(v);   // row_shr:4
  v += dpp_movf<0x118>(v);   // row_shr:8
  const auto rl = [&](int lane) { return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane)); };
  return (rl(12) + rl(29)) + (rl(46) + rl(63));
}

// log x = k log 2 + log m for a positive double x: k (returned in kk, an integer-valued double)
// and log m, m = x 2^-k in [1/sqrt 2, sqrt 2), from log m = 2 atanh(z), z = (m - 1) / (m + 1),
// |z| <= 0.1716, with the odd series of atanh summed to z^19 (the first omitted term is below
// 1e-17).  m - 1 is exact, so log m is accurate to a few units in the last place.  A NaN or
// infinite x gives a NaN.
__device__ __forceinline__ double log_split(double x, double& kk) {
  int k = __builtin_amdgcn_frexp_exp(x);          // x = m 2^k, m in [0.5, 1)
  double m = __builtin_amdgcn_frexp_mant(x);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    --k;
  }
  kk = (double)k;
  const double z = (m - 1.0) / (m + 1.0), z2 = z * z;
  double p = 1.0 / 19;
  p = fma(p, z2, 1.0 / 17);
  p = fma(p, z2, 1.0 / 15);
  p = fma(p, z2, 1.0 / 13);
  p = fma(p, z2, 1.0 / 11);
  p = fma(p, z2, 1.0 / 9);
  p = fma(p, z2, 1.0 / 7);
  p = fma(p, z2, 1.0 / 5);
  p = fma(p, z2, 1.0 / 3);
  p = fma(p, z2, 1.0);
  return 2.0 * z * p;
}

// Diagonal updates v + a of a diagonal block: for the real 16 x 16 case (registers to spare at
// full occupancy) as fma(a, dg[r], v) with a per-lane 0.0 / 1.0 indicator, one instruction; in
// the other cases as a lane select, which keeps the indicator out of the registers.
template <int NB, bool CPLX>
struct XDiag {
  static constexpr bool kFma = NB == 1 && !CPLX;
  double dg[kFma ? 4 : 1];
  int l;
  __device__ __forceinline__ explicit XDiag(int lane) : l(lane) {
    if constexpr (kFma) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dg[r] = xdiag(r, lane) ? 1.0 : 0.0;
    }
  }
  __device__ __forceinline__ double add(int r, double a, double v) const {
    if constexpr (kFma) return fma(a, dg[r], v);   // exactly v off the diagonal
    else return xdiag(r, l) ? v + a : v;
  }
};

// D = a I + b A + c A2 (+ d A3)
template <int NB, bool CPLX, bool WITH3>
__device__ __forceinline__ void xpoly(XMat<NB, CPLX>& D, double a, double b, double c, double d,
                                      const XMat<NB, CPLX>& A1, const XMat<NB, CPLX>& A2,
                                      const XMat<NB, CPLX>& A3, const XDiag<NB, CPLX>& dg) {
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = fma(c, A2.re[I][J][r], b * A1.re[I][J][r]);
        if constexpr (WITH3) v = fma(d, A3.re[I][J][r], v);
        if (I == J) v = dg.add(r, a, v);
        D.re[I][J][r] = v;
        if constexpr (CPLX) {
          double w = fma(c, A2.im[I][J][r], b * A1.im[I][J][r]);
          if constexpr (WITH3) w = fma(d, A3.im[I][J][r], w);
          D.im[I][J][r] = w;
        }
      }
}

template <typename T, bool CPLX, int DE>
__global__ __launch_bounds__(64) void k_cluster_expm(ClusterArgs<T> A) {
  constexpr int LD = DE + 1;
  constexpr int NB = DE / 16;
  __shared__ T sar[DE * LD];
  __shared__ T sai[CPLX ? DE * LD : 1];
  const int64_t c = xcd_cluster(blockIdx.x, A.n);
  const int l = threadIdx.x;
  const T th = A.tab ? (T)A.tab->theta_cur : (T)A.theta;
  const double beta = A.tab ? A.tab->beta : A.beta;
  constexpr int NBITS = log2i(DE);
  static_assert(NBITS == 4 || NBITS == 5, "the one-wave kernel covers D = 16 and 32");
  const int Dc = A.Dc;
  const int nch = A.maxch;
  const bool lut = nch <= kExpmLut;   // cluster-uniform
  // per child: pext of every cluster index onto the child's sites, and pdep of (child index a,
  // complement index x) back to the cluster index, as LDS tables
  __shared__ unsigned char pextL[kExpmLut][DE], depL[kExpmLut][DE];
  __shared__ T stc_r[kExpmLut][DE * DE / 4];
  __shared__ T stc_i[CPLX ? kExpmLut : 1][CPLX ? DE * DE / 4 : 1];
  XMat<NB, CPLX> X, P2, P3, M;
  // ---- a1/a2: assemble theta_e at eta ----
  // D_c and D_e / D_c are powers of two: shifts and masks instead of integer division
  const int ldc = Dc > 0 ? __builtin_ctz(Dc) : 0;
  const int lnr = NBITS - ldc;
  if (lut) {
    for (int s = 0; s < nch; ++s) {
      const int mask = A.chmask[(int64_t)s * A.n + c] & (DE - 1);
      if (l < DE) {
        pextL[s][l] = kSiteBits.pext[mask][l];
        if constexpr (NBITS == 4) depL[s][l] = kSiteBits.pdep4[mask][l];
        else depL[s][l] = kSiteBits.pdep5[mask][l];
      }
    }
    __syncthreads();
    // branch-free element assembly: every candidate element is loaded from a valid address and
    // then selected, so the lanes of the wave never diverge
    // (h_e, then the children in slot order, then the parents: the order of the generic path)
    const int64_t ho = A.hoff[c];
    T acr[NB][NB][4], aci[NB][NB][4];
    // h_e from its packed upper triangle (real plane, then the strict upper imaginary plane);
    // the cluster-uniform test sits outside the loop so that a lane's loads issue together.  The
    // packed index of (lo, hi), lo <= hi, is lo (2D + 1 - lo) / 2 + hi - lo, and the strict one
    // lo (2D - 1 - lo) / 2 + hi - lo - 1; both products are even.
    if (ho >= 0) {
      const double* hp = A.h + ho;
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * I + 4 * r + (l >> 4), j = 16 * J + (l & 15);
            const unsigned lo = (unsigned)min(i, j), hi = (unsigned)max(i, j);
            acr[I][J][r] = (T)hp[((lo * (2u * DE + 1u - lo)) >> 1) + hi - lo];
            if constexpr (CPLX) {
              const double v = hp[DE * (DE + 1) / 2 + (lo < hi ? ((lo * (2u * DE - 1u - lo)) >> 1) + hi - lo - 1u : 0u)];
              aci[I][J][r] = (T)(i < j ? v : (i > j ? -v : 0.0));
            } else {
              aci[I][J][r] = T(0);
            }
          }
    } else {
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acr[I][J][r] = T(0);
            aci[I][J][r] = T(0);
          }
    }
    // the (extrapolated) child messages, dense D_c x D_c in LDS, one pass over all children
    for (int idx = l; idx < nch << (2 * ldc); idx += 64) {
      const int s = idx >> (2 * ldc), ab = idx & ((1 << (2 * ldc)) - 1);
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int a = ab >> ldc, b = ab & (Dc - 1);
      T er, ei;
      if (A.ze_c)
        herm_elem_bf<T, CPLX>([&](int k) { const int64_t o = (int64_t)k * A.Mc + m;
                                           return extrap<T>(A.nu_c[o], A.ze_c[o], th); }, a, b, Dc, er, ei);
      else
        herm_elem_bf<T, CPLX>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, a, b, Dc, er, ei);
      stc_r[s][ab] = er;
      if constexpr (CPLX) stc_i[s][ab] = ei;
    }
    __syncthreads();
    for (int s = 0; s < nch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;   // cluster-uniform
      const int mask = A.chmask[(int64_t)s * A.n + c];
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * I + 4 * r + (l >> 4), j = 16 * J + (l & 15);
            const bool ok = ((i ^ j) & ~mask & (DE - 1)) == 0;
            const int ab = (pextL[s][i] << ldc) | pextL[s][j];
            acr[I][J][r] -= ok ? stc_r[s][ab] : T(0);
            if constexpr (CPLX) aci[I][J][r] -= ok ? stc_i[s][ab] : T(0);
          }
    }
    for (int s = 0; s < A.maxpar; ++s) {
      const int m = A.par[(int64_t)s * A.n + c];
      if (m < 0) continue;   // cluster-uniform
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * I + 4 * r + (l >> 4), j = 16 * J + (l & 15);
            T er, ei;
            if (A.ze_p)
              herm_elem_bf<T, CPLX>([&](int k) { const int64_t o = (int64_t)k * A.Mp + m;
                                                 return extrap<T>(A.nu_p[o], A.ze_p[o], th); }, i, j, DE, er, ei);
            else
              herm_elem_bf<T, CPLX>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, i, j, DE, er, ei);
            acr[I][J][r] += er;
            aci[I][J][r] += ei;
          }
    }
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          X.re[I][J][r] = (double)acr[I][J][r];
          if constexpr (CPLX) X.im[I][J][r] = (double)aci[I][J][r];
        }
  } else {
    lds_assemble<T, CPLX, DE, 64>(A, c, l, A.nu_c, A.ze_c, A.nu_p, A.ze_p, th, true, T(1), sar, sai);
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * I + 4 * r + (l >> 4)) * LD + 16 * J + (l & 15);
          X.re[I][J][r] = (double)sar[o];
          if constexpr (CPLX) X.im[I][J][r] = (double)sai[o];
        }
  }
  // ---- shift, scale ----
  const double mu = xtrace(X, l) / DE;
  const XDiag<NB, CPLX> dg(l);
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) X.re[I][I][r] = dg.add(r, -mu, X.re[I][I][r]);
  // The scale uses the induced 1-norm, an upper bound of the spectral radius: the largest column
  // sum (theta is Hermitian, so it equals the largest row sum).  Column 16 J + l%16 of block
  // column J is spread over the registers of the lanes l%16 + 16 g; two xor-shuffles complete it
  // in every lane, a DPP row maximum then leaves the largest column sum in every lane.  (On these
  // clusters it is at most the Frobenius norm, the other bound at hand, so that one is not
  // formed; moduli of complex entries use the hardware square root, as nrm only chooses s.)
  double rmax = 0.0;
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    double a = 0.0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (CPLX) a += __builtin_amdgcn_sqrt(fma(X.re[I][J][r], X.re[I][J][r], X.im[I][J][r] * X.im[I][J][r]));
        else a += fabs(X.re[I][J][r]);
      }
    a += __shfl_xor(a, 16, 64);
    a += __shfl_xor(a, 32, 64);
    rmax = fmax(rmax, a);
  }
  rmax = fmax(rmax, dpp_mov<0xB1>(rmax));    // quad_perm [1, 0, 3, 2]
  rmax = fmax(rmax, dpp_mov<0x4E>(rmax));    // quad_perm [2, 3, 0, 1]
  rmax = fmax(rmax, dpp_mov<0x141>(rmax));   // row_half_mirror
  rmax = fmax(rmax, dpp_mov<0x140>(rmax));   // row_mirror
  const double nrm = beta * rmax;
  // s = the least s >= 0 with nrm <= 2^(s-1), at most 200 (0 for a NaN norm): from the binary
  // exponent of nrm instead of a search
  int s;
  if (!(nrm > 0.5)) {
    s = 0;
  } else if (!(nrm <= 0x1p199)) {
    s = 200;
  } else {
    int e;
    const double m = frexp(nrm, &e);   // nrm = m 2^e, 0.5 <= m < 1
    s = m == 0.5 ? e : e + 1;
  }
  s = __builtin_amdgcn_readfirstlane(s);   // every lane holds the same value; make it scalar
  const double sc = -ldexp(beta, -s);
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        X.re[I][J][r] *= sc;
        if constexpr (CPLX) X.im[I][J][r] *= sc;
      }
  // ---- E0 = T_m(X): powers X^2, X^3 and a Horner recursion in X^3 ----
  // m = 12 for double messages.  Float messages take m = 8 (one product fewer): for ||X|| <= 1/2
  // the truncation is below 0.5^9 / 9! = 5.4e-9, a backward error on X under 0.2 u_32 relative,
  // below what the FP32 squarings and the float rounding of the messages already put there.
  constexpr double c0 = 1.0, c1 = 1.0, c2 = 1.0 / 2, c3 = 1.0 / 6, c4 = 1.0 / 24, c5 = 1.0 / 120,
                   c6 = 1.0 / 720, c7 = 1.0 / 5040, c8 = 1.0 / 40320, c9 = 1.0 / 362880, c10 = 1.0 / 3628800,
                   c11 = 1.0 / 39916800, c12 = 1.0 / 479001600;
  constexpr bool kDeg8 = std::is_same<T, float>::value;
  xzero(P2);
  xmm(X, X, P2);
  xzero(P3);
  xmm(X, P2, P3);
  if constexpr (kDeg8) xpoly<NB, CPLX, false>(M, c6, c7, c8, 0.0, X, P2, P3, dg);    // B2
  else xpoly<NB, CPLX, true>(M, c9, c10, c11, c12, X, P2, P3, dg);                  // B3
  {
    XMat<NB, CPLX> B;
    if constexpr (!kDeg8) {
      xpoly<NB, CPLX, false>(B, c6, c7, c8, 0.0, X, P2, P3, dg);   // B2 + X^3 B3
      xmm(P3, M, B);
      M = B;
    }
    xpoly<NB, CPLX, false>(B, c3, c4, c5, 0.0, X, P2, P3, dg);   // B1 + X^3 (...)
    xmm(P3, M, B);
    M = B;
    xpoly<NB, CPLX, false>(B, c0, c1, c2, 0.0, X, P2, P3, dg);   // B0 + X^3 (...)
    xmm(P3, M, B);
    M = B;
  }
  // ---- normalise and square s times ----
  // Every rescaling is by an exact power of two 2^-e_j, e_j the binary exponent of the trace
  // (frexp's exponent minus one; a non-finite trace leaves the result non-finite, which is flagged):
  // first E0 itself (e_0, so Y_0 has trace in [1, 2)), then the squares j = 3, 7, 11, ...  For a
  // PSD Y with trace at least 1 the largest eigenvalue is at least 1/D, so four unscaled
  // squarings keep the trace within [D^-16, 2^16], far inside the FP32 and FP64 ranges, and up to
  // three more after the last rescaling keep it above D^-8.  The exponents are accumulated as an
  // integer, E <- 2E + e_j (starting from E = e_0), so no logarithm or division sits in the loop:
  //     log Z = E log 2 + log Tr Y_s,   rho = Y_s / Tr Y_s.
  // X and M alternate as product buffers (the loop is unrolled by two).
  // E holds the accumulated exponent as of squaring jr (jr = -1: before the first); the value
  // after squaring j is E 2^(j - jr), so only the rescaling points touch it (ldexp is exact here).
  double E;
  int jr = -1;
  {
    const int e0 = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_frexp_expf(xtrace_est(M, l)) - 1);
    E = (double)e0;
    const double sc0 = ldexp(1.0, -e0);
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          M.re[I][J][r] *= sc0;
          if constexpr (CPLX) M.im[I][J][r] *= sc0;
        }
  }
  // Float messages: the squarings after the first kF64Squarings (up to and including the
  // rescaling at j = 3) run on the FP32 matrix cores.  A relative rounding error e in Y_j acts on rho
  // like an error of about 2^(s-j) e in X = beta (theta - mu), and 2^s is about 2 ||X||, so for
  // j >= 4 the float squarings perturb X by at most about ||X|| u_32 / 8 times the product's error
  // growth, the order of what the float rounding of the messages themselves puts on X
  // (beta ||nu|| u_32).  The polynomial and the first squarings, where the error would be
  // amplified most, stay in FP64.
  int n64 = s;
  if constexpr (std::is_same<T, float>::value) n64 = s < kF64Squarings ? s : kF64Squarings;
  auto post = [&](XMat<NB, CPLX>& Y, int j) {
    if ((j & 3) == 3) {
      const int e = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_frexp_expf(xtrace_est(Y, l)) - 1);
      E = ldexp(E, j - jr) + (double)e;
      jr = j;
      const double sc2 = ldexp(1.0, -e);
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            Y.re[I][J][r] *= sc2;
            if constexpr (CPLX) Y.im[I][J][r] *= sc2;
          }
    }
  };
  for (int j = 0; j < n64; j += 2) {
    xzero(X);
    xmm(M, M, X);
    post(X, j);
    if (j + 1 < n64) {
      xzero(M);
      xmm(X, X, M);
      post(M, j + 1);
    } else {
      M = X;
    }
  }
  if (n64 < s) {
    // to the FP32 layout through LDS, squarings n64 .. s-1, and back
    XMat32<NB, CPLX> Ya, Yb;
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * I + 4 * r + (l >> 4)) * LD + 16 * J + (l & 15);
          sar[o] = (T)M.re[I][J][r];
          if constexpr (CPLX) sai[o] = (T)M.im[I][J][r];
        }
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * I + 4 * (l >> 4) + r) * LD + 16 * J + (l & 15);
          Ya.re[I][J][r] = (float)sar[o];
          if constexpr (CPLX) Ya.im[I][J][r] = (float)sai[o];
        }
    auto post32 = [&](XMat32<NB, CPLX>& Y, int j) {
      if ((j & 3) == 3) {
        const int e = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_frexp_expf(xtrace32(Y, l)) - 1);
        E = ldexp(E, j - jr) + (double)e;
        jr = j;
        const float sc2 = ldexpf(1.f, -e);
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = 0; J < NB; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              Y.re[I][J][r] *= sc2;
              if constexpr (CPLX) Y.im[I][J][r] *= sc2;
            }
      }
    };
    for (int j = n64; j < s; j += 2) {
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            Yb.re[I][J][r] = 0.f;
            if constexpr (CPLX) Yb.im[I][J][r] = 0.f;
          }
      xmm32(Ya, Ya, Yb);
      post32(Yb, j);
      if (j + 1 < s) {
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = 0; J < NB; ++J)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              Ya.re[I][J][r] = 0.f;
              if constexpr (CPLX) Ya.im[I][J][r] = 0.f;
            }
        xmm32(Yb, Yb, Ya);
        post32(Ya, j + 1);
      } else {
        Ya = Yb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * I + 4 * (l >> 4) + r) * LD + 16 * J + (l & 15);
          sar[o] = (T)Ya.re[I][J][r];
          if constexpr (CPLX) sai[o] = (T)Ya.im[I][J][r];
        }
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (16 * I + 4 * r + (l >> 4)) * LD + 16 * J + (l & 15);
          M.re[I][J][r] = (double)sar[o];
          if constexpr (CPLX) M.im[I][J][r] = (double)sai[o];
        }
  }
  double L;
  {
    E = ldexp(E, s - 1 - jr);   // the exponent after the last squaring
    const double tf = xtrace(M, l);
    double kf;
    const double lm = log_split(tf, kf);
    L = fma(E + kf, 0.69314718055994530942, lm);   // E + kf is exact
    // 1 / tf from the hardware reciprocal and two Newton steps (tf is a positive normal number)
    double it = __builtin_amdgcn_rcp(tf);
    it = fma(fma(-tf, it, 1.0), it, it);
    it = fma(fma(-tf, it, 1.0), it, it);
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          M.re[I][J][r] *= it;
          if constexpr (CPLX) M.im[I][J][r] *= it;
        }
  }
  const double F = mu - L / beta;
  const int32_t gid = A.gid[c];
  if (l == 0) {
    if (A.scal) A.scal[gid] = F;
    if (!isfinite(F) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  }
  // ---- a5: rho back to LDS, then the outputs ----
  __syncthreads();
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (16 * I + 4 * r + (l >> 4)) * LD + 16 * J + (l & 15);
        sar[o] = (T)M.re[I][J][r];
        if constexpr (CPLX) sai[o] = (T)M.im[I][J][r];
      }
  __syncthreads();
  if (!lut) {
    lds_outputs<T, CPLX, DE, 64>(A, c, l, gid, sar, sai);
    return;
  }
  // own marginal slot and per-cluster marginal, straight from the registers (upper triangle)
  const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
  if ((rs_self >= 0 && A.R) || A.marg) {
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + 4 * r + (l >> 4), j = 16 * J + (l & 15);
          if (i > j) continue;
          const int kr = tri_index(i, j, DE);
          const T vr = (T)M.re[I][J][r];
          if (rs_self >= 0 && A.R) A.R[(int64_t)kr * A.S + rs_self] = vr;
          if (A.marg) A.marg[A.marg_off[gid] + kr] = vr;
          if constexpr (CPLX) {
            if (i < j) {
              const int ki = DE * (DE + 1) / 2 + stri_index(i, j, DE);
              const T vi = (T)M.im[I][J][r];
              if (rs_self >= 0 && A.R) A.R[(int64_t)ki * A.S + rs_self] = vi;
              if (A.marg) A.marg[A.marg_off[gid] + ki] = vi;
            }
          }
        }
  }
  // partial traces onto every child, all (child, component) pairs across the lanes
  if (A.Tout && Dc > 0) {
    const int NR = 1 << lnr;
    const int NCC = CPLX ? Dc * Dc : Dc * (Dc + 1) / 2;
    for (int idx = l; idx < nch * NCC; idx += 64) {
      int s = 0, k = idx;
      while (k >= NCC) {   // (child, component) without an integer division; at most nch steps
        k -= NCC;
        ++s;
      }
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      int a, b;
      bool im;
      decode_comp(k, Dc, a, b, im);
      const T* y = im ? sai : sar;
      T sum = T(0);
      for (int x = 0; x < NR; ++x) sum += y[depL[s][(a << lnr) + x] * LD + depL[s][(b << lnr) + x]];
      A.Tout[(int64_t)k * A.Mc + m] = sum;
    }
  }
}

// Workgroup variant for De = 32 (complex), 64, 128, 256: five matrices (X, X^2, X^3 and two Horner / squaring
// buffers) in a per-workgroup FP64 slab, row-major, real plane then imaginary plane; four
// waves, each computing 32 x 32 output tiles (2 x 2 blocks of the 16 x 16 MFMA; 16 x 16 below De = 128).  The A operand
// of block (I, K) is read as the conjugate of block (K, I), which keeps both operand reads as
// rows of 16 consecutive doubles.
struct GInit {
  double a, b, c;             // C = a I + b X + c P + scale * (A B)
  const double* xr; const double* xi;
  const double* pr; const double* pi;
};

template <bool CPLX, int DE>
__device__ double gmm(const double* xr, const double* xi, const double* yr, const double* yi, double* cr_,
                      double* ci_, double scale, const GInit& in, int tid) {
  constexpr int TB = DE >= 128 ? 2 : 1;   // output tile of TB x TB blocks per wave
  constexpr int NB = DE / 16, NT = NB / TB;
  const int wave = tid / 64, l = tid % 64;
  const int lr = l >> 4, lc = l & 15;
  double tr = 0.0;
  // C is Hermitian (every product here is a polynomial in one matrix): only the tiles on and
  // above the diagonal are computed, an off-diagonal tile is also written conjugate-transposed
  for (int t = wave; t < NT * (NT + 1) / 2; t += 4) {
    int TI = 0, TJ = t;
    while (TJ >= NT - TI) {
      TJ -= NT - TI;
      ++TI;
    }
    TJ += TI;
    mfma_f64x4 accr[TB][TB], acci[TB][TB];
#pragma unroll
    for (int ii = 0; ii < TB; ++ii)
#pragma unroll
      for (int jj = 0; jj < TB; ++jj) {
        accr[ii][jj] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
        acci[ii][jj] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
      }
    // operand fragments of one K step (four k-sub-steps); with 16 x 16 tiles they are loaded one
    // step ahead of the products that use them, so the L2 latency overlaps the matrix-core work
    constexpr int NP = CPLX ? 2 : 1;
    double fa[2][4][TB][NP], fb[2][4][TB][NP];
    auto load_step = [&](int K, double (&ga)[4][TB][NP], double (&gb)[4][TB][NP]) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int64_t row = (int64_t)(16 * K + 4 * kk + lr) * DE;
#pragma unroll
        for (int q = 0; q < TB; ++q) {
          const int ca = 16 * (TB * TI + q) + lc, cb = 16 * (TB * TJ + q) + lc;
          ga[kk][q][0] = xr[row + ca];
          gb[kk][q][0] = yr[row + cb];
          if constexpr (CPLX) {
            ga[kk][q][1] = xi[row + ca];
            gb[kk][q][1] = yi[row + cb];
          }
        }
      }
    };
    auto mma_step = [&](const double (&ga)[4][TB][NP], const double (&gb)[4][TB][NP]) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int ii = 0; ii < TB; ++ii)
#pragma unroll
          for (int jj = 0; jj < TB; ++jj) {
            accr[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[kk][ii][0], gb[kk][jj][0], accr[ii][jj], 0, 0, 0);
            if constexpr (CPLX) {
              accr[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[kk][ii][1], gb[kk][jj][1], accr[ii][jj], 0, 0, 0);
              acci[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[kk][ii][0], gb[kk][jj][1], acci[ii][jj], 0, 0, 0);
              acci[ii][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[kk][ii][1], gb[kk][jj][0], acci[ii][jj], 0, 0, 0);
            }
          }
    };
    if constexpr (TB == 1) {   // 16 x 16 tiles: latency-bound, registers to spare
      load_step(0, fa[0], fb[0]);
#pragma unroll 1
      for (int K = 0; K < NB; K += 2) {
        if (K + 1 < NB) load_step(K + 1, fa[1], fb[1]);
        mma_step(fa[0], fb[0]);
        if (K + 1 < NB) {
          if (K + 2 < NB) load_step(K + 2, fa[0], fb[0]);
          mma_step(fa[1], fb[1]);
        }
      }
    } else {
      // 32 x 32 tiles: one K step at a time.  Its 32 loads in flight together hide the latency
      // better than a ring of k-sub-step fragments loaded two or three k-sub-steps ahead (30 %
      // slower at D = 128 and 256), and a second K-step buffer costs the second wave per SIMD.
#pragma unroll 1
      for (int K = 0; K < NB; ++K) {
        load_step(K, fa[0], fb[0]);
        mma_step(fa[0], fb[0]);
      }
    }
#pragma unroll
    for (int ii = 0; ii < TB; ++ii)
#pragma unroll
      for (int jj = 0; jj < TB; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * (TB * TI + ii) + 4 * r + lr, j = 16 * (TB * TJ + jj) + lc;
          const int64_t o = (int64_t)i * DE + j;
          double vr = scale * accr[ii][jj][r];
          if (in.b != 0.0) vr = fma(in.b, in.xr[o], vr);
          if (in.c != 0.0) vr = fma(in.c, in.pr[o], vr);
          if (i == j) {
            vr += in.a;
            tr += vr;
          }
          cr_[o] = vr;
          const int64_t ot = (int64_t)j * DE + i;
          if (TI != TJ) cr_[ot] = vr;
          if constexpr (CPLX) {
            double vi = scale * acci[ii][jj][r];
            if (in.b != 0.0) vi = fma(in.b, in.xi[o], vi);
            if (in.c != 0.0) vi = fma(in.c, in.pi[o], vi);
            ci_[o] = (i == j) ? 0.0 : vi;
            if (TI != TJ) ci_[ot] = -vi;
          }
        }
  }
  return tr;
}

// C = scale (Y Y) for Hermitian Y in FP32 (the float-message path's later squarings): gmm's tiling
// and operand reads on FP32 slabs with v_mfma_f32_16x16x4_f32, whose operands are laid out like
// the FP64 instruction's and whose result register r of lane l holds row 4 (l/16) + r.  Returns
// this thread's share of the trace.
template <bool CPLX, int DE>
__device__ double gsq32(const float* yr, const float* yi, float* cr_, float* ci_, float scale, int tid) {
  constexpr int TB = DE >= 128 ? 2 : 1;
  constexpr int NB = DE / 16, NT = NB / TB;
  constexpr int NP = CPLX ? 2 : 1;
  const int wave = tid / 64, l = tid % 64;
  const int lr = l >> 4, lc = l & 15;
  double tr = 0.0;
  for (int t = wave; t < NT * (NT + 1) / 2; t += 4) {
    int TI = 0, TJ = t;
    while (TJ >= NT - TI) {
      TJ -= NT - TI;
      ++TI;
    }
    TJ += TI;
    mfma_f32x4 accr[TB][TB], acci[TB][TB];
#pragma unroll
    for (int ii = 0; ii < TB; ++ii)
#pragma unroll
      for (int jj = 0; jj < TB; ++jj) {
        accr[ii][jj] = mfma_f32x4{0.f, 0.f, 0.f, 0.f};
        acci[ii][jj] = mfma_f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll 1
    for (int K = 0; K < NB; ++K) {
      float ga[4][TB][NP], gb[4][TB][NP];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int64_t row = (int64_t)(16 * K + 4 * kk + lr) * DE;
#pragma unroll
        for (int q = 0; q < TB; ++q) {
          const int ca = 16 * (TB * TI + q) + lc, cb = 16 * (TB * TJ + q) + lc;
          ga[kk][q][0] = yr[row + ca];
          gb[kk][q][0] = yr[row + cb];
          if constexpr (CPLX) {
            ga[kk][q][1] = yi[row + ca];
            gb[kk][q][1] = yi[row + cb];
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int ii = 0; ii < TB; ++ii)
#pragma unroll
          for (int jj = 0; jj < TB; ++jj) {
            accr[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[kk][ii][0], gb[kk][jj][0], accr[ii][jj], 0, 0, 0);
            if constexpr (CPLX) {
              accr[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[kk][ii][1], gb[kk][jj][1], accr[ii][jj], 0, 0, 0);
              acci[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[kk][ii][0], gb[kk][jj][1], acci[ii][jj], 0, 0, 0);
              acci[ii][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ga[kk][ii][1], gb[kk][jj][0], acci[ii][jj], 0, 0, 0);
            }
          }
    }
#pragma unroll
    for (int ii = 0; ii < TB; ++ii)
#pragma unroll
      for (int jj = 0; jj < TB; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * (TB * TI + ii) + 4 * lr + r, j = 16 * (TB * TJ + jj) + lc;
          const int64_t o = (int64_t)i * DE + j;
          const float vr = scale * accr[ii][jj][r];
          if (i == j) tr += vr;
          cr_[o] = vr;
          const int64_t ot = (int64_t)j * DE + i;
          if (TI != TJ) cr_[ot] = vr;
          if constexpr (CPLX) {
            const float vi = scale * acci[ii][jj][r];
            ci_[o] = (i == j) ? 0.f : vi;
            if (TI != TJ) ci_[ot] = -vi;
          }
        }
  }
  return tr;
}

template <typename T, bool CPLX, int DE>
__global__ __launch_bounds__(256) void k_cluster_expm_wg(ClusterArgs<T> A, double* scratch, int64_t slab) {
  constexpr int64_t DD = (int64_t)DE * DE;
  constexpr int NPL = CPLX ? 2 : 1;
  __shared__ double red[8];
  const int tid = threadIdx.x, nth = blockDim.x;
  double* base = scratch + (int64_t)blockIdx.x * slab;
  double* mr[5];
  double* mi[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    mr[k] = base + (int64_t)k * NPL * DD;
    mi[k] = CPLX ? mr[k] + DD : nullptr;
  }
  double *Xr = mr[0], *Xi = mi[0], *P2r = mr[1], *P2i = mi[1], *P3r = mr[2], *P3i = mi[2];
  const T th = A.tab ? (T)A.tab->theta_cur : (T)A.theta;
  const double beta = A.tab ? A.tab->beta : A.beta;
  constexpr double c0 = 1.0, c1 = 1.0, c2 = 1.0 / 2, c3 = 1.0 / 6, c4 = 1.0 / 24, c5 = 1.0 / 120,
                   c6 = 1.0 / 720, c7 = 1.0 / 5040, c8 = 1.0 / 40320, c9 = 1.0 / 362880, c10 = 1.0 / 3628800,
                   c11 = 1.0 / 39916800, c12 = 1.0 / 479001600;
  const GInit zero{0.0, 0.0, 0.0, nullptr, nullptr, nullptr, nullptr};
  for (int64_t c = blockIdx.x; c < A.n; c += gridDim.x) {
    double *Mr = mr[3], *Mi = mi[3], *Br = mr[4], *Bi = mi[4];
    // ---- a1/a2: assemble theta_e at eta ----
    big_assemble<T, double, CPLX, false>(A, c, DE, Xr, Xi, (double*)nullptr, (double*)nullptr, th, tid, nth);
    __syncthreads();
    // ---- shift and scale: X = -(beta / 2^s) (theta - mu) ----
    double tr = 0.0;
    for (int k = tid; k < DE; k += nth) tr += Xr[(int64_t)k * DE + k];
    const double mu = block_sum(tr, red) / DE;
    double n2 = 0.0;
    for (int64_t idx = tid; idx < DD; idx += nth) {
      const double v = Xr[idx] - ((idx / DE == idx % DE) ? mu : 0.0);
      n2 = fma(v, v, n2);
      if constexpr (CPLX) n2 = fma(Xi[idx], Xi[idx], n2);
    }
    double rmax = 0.0;   // induced 1-norm: one row per thread
    for (int i = tid; i < DE; i += nth) {
      const double* xr = Xr + (int64_t)i * DE;
      double a = 0.0;
      for (int j = 0; j < DE; ++j) {
        const double v = xr[j] - (i == j ? mu : 0.0);
        if constexpr (CPLX) a += sqrt(fma(v, v, Xi[(int64_t)i * DE + j] * Xi[(int64_t)i * DE + j]));
        else a += fabs(v);
      }
      rmax = fmax(rmax, a);
    }
    const double nrm = beta * fmin(sqrt(block_sum(n2, red)), block_max(rmax, red));
    int s = 0;
    while (s < 200 && nrm > ldexp(0.5, s)) ++s;   // block-uniform
    const double sc = -ldexp(beta, -s);
    for (int64_t idx = tid; idx < DD; idx += nth) {
      Xr[idx] = sc * (Xr[idx] - ((idx / DE == idx % DE) ? mu : 0.0));
      if constexpr (CPLX) Xi[idx] *= sc;
    }
    __syncthreads();
    // ---- E0 = T_m(X): m = 12, or 8 for float messages (one product fewer; see k_cluster_expm) ----
    constexpr bool kDeg8 = std::is_same<T, float>::value;
    gmm<CPLX, DE>(Xr, Xi, Xr, Xi, P2r, P2i, 1.0, zero, tid);
    __syncthreads();
    gmm<CPLX, DE>(Xr, Xi, P2r, P2i, P3r, P3i, 1.0, zero, tid);
    __syncthreads();
    for (int64_t idx = tid; idx < DD; idx += nth) {
      const bool diag = idx / DE == idx % DE;
      if constexpr (kDeg8) {
        Mr[idx] = fma(c8, P2r[idx], c7 * Xr[idx]) + (diag ? c6 : 0.0);
        if constexpr (CPLX) Mi[idx] = fma(c8, P2i[idx], c7 * Xi[idx]);
      } else {
        Mr[idx] = fma(c12, P3r[idx], fma(c11, P2r[idx], c10 * Xr[idx])) + (diag ? c9 : 0.0);
        if constexpr (CPLX) Mi[idx] = fma(c12, P3i[idx], fma(c11, P2i[idx], c10 * Xi[idx]));
      }
    }
    __syncthreads();
    const double hc[3][3] = {{c6, c7, c8}, {c3, c4, c5}, {c0, c1, c2}};
    double trp = 0.0;
    for (int h = kDeg8 ? 1 : 0; h < 3; ++h) {
      const GInit in{hc[h][0], hc[h][1], hc[h][2], Xr, Xi, P2r, P2i};
      trp = gmm<CPLX, DE>(P3r, P3i, Mr, Mi, Br, Bi, 1.0, in, tid);
      __syncthreads();
      double* tp = Mr; Mr = Br; Br = tp;
      tp = Mi; Mi = Bi; Bi = tp;
    }
    // ---- normalise and square: Z_{j+1} = Z_j^2 / (Tr Z_j)^2 ----
    // (float messages: the squarings after the first kF64Squarings in FP32, in the buffers of X^2
    // and X^3, which the polynomial no longer needs; see k_cluster_expm)
    double t = block_sum(trp, red);
    double L = log(t);
    const int n64 = std::is_same<T, float>::value ? (s < kF64Squarings ? s : kF64Squarings) : s;
    for (int j = 0; j < n64; ++j) {
      trp = gmm<CPLX, DE>(Mr, Mi, Mr, Mi, Br, Bi, 1.0 / (t * t), zero, tid);
      __syncthreads();
      double* tp = Mr; Mr = Br; Br = tp;
      tp = Mi; Mi = Bi; Bi = tp;
      t = block_sum(trp, red);
      L = fma(2.0, L, log(t));
    }
    if (n64 < s) {
      float* fa_r = reinterpret_cast<float*>(P2r);
      float* fa_i = CPLX ? fa_r + DD : nullptr;
      float* fb_r = fa_r + NPL * DD;
      float* fb_i = CPLX ? fb_r + DD : nullptr;
      for (int64_t idx = tid; idx < DD; idx += nth) {
        fa_r[idx] = (float)Mr[idx];
        if constexpr (CPLX) fa_i[idx] = (float)Mi[idx];
      }
      __syncthreads();
      for (int j = n64; j < s; ++j) {
        trp = gsq32<CPLX, DE>(fa_r, fa_i, fb_r, fb_i, (float)(1.0 / (t * t)), tid);
        __syncthreads();
        float* tp = fa_r; fa_r = fb_r; fb_r = tp;
        tp = fa_i; fa_i = fb_i; fb_i = tp;
        t = block_sum(trp, red);
        L = fma(2.0, L, log(t));
      }
      for (int64_t idx = tid; idx < DD; idx += nth) {
        Mr[idx] = (double)fa_r[idx];
        if constexpr (CPLX) Mi[idx] = (double)fa_i[idx];
      }
      __syncthreads();
    }
    const double F = mu - L / beta;
    const int32_t gid = A.gid[c];
    if (tid == 0) {
      if (A.scal) A.scal[gid] = F;
      if (!isfinite(F) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
    }
    // ---- a5: outputs of rho = Z_s / Tr Z_s ----
    big_outputs<T, double, CPLX>(A, c, DE, gid, Mr, Mi, 1.0 / t, tid, nth);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// certified lambda_min for De >= 64 without eigenvectors (a8)
// ------------------------------------------------------------------------------------------
//
// theta_e (FP64, in a per-workgroup slab) is reduced to a Hermitian tridiagonal matrix by De - 2
// Householder reflections H = I - tau v v^H acting on the trailing block (A <- H A H with the
// rank-2 form A - v w^H - w v^H, w = p - (tau/2)(v^H p) v, p = tau A v).  A diagonal unitary
// makes the off-diagonal real and non-negative, so the eigenvalues are those of the real
// symmetric tridiagonal (d, |e|).  lambda_min is then bracketed by multisection on Sturm counts
// (number of eigenvalues below x from the signs of the LDL^T pivots), 256 points per round;
// the lower end of the final bracket, below which no eigenvalue lies, is returned.
template <bool CPLX, int DE>
__device__ void tridiag_lambda_min(const ClusterArgs<double>& A, int64_t c, double* ar, double* ai, double nrm2) {
  __shared__ double vr[DE], vi[DE], pr[DE], pi[DE];
  __shared__ double qvr[DE], qvi[DE], qwr[DE], qwi[DE];
  __shared__ double dg[DE], e2[DE];
  __shared__ double red[16];
  const int tid = threadIdx.x, nth = blockDim.x;
  {
    // The rank-2 update of each reflection is applied during the next reflection's sweep over
    // the trailing matrix (pending vectors qv, qw): every trailing element is read and written
    // once per reflection instead of read twice and written once.  Row k and the final 2 x 2
    // block are corrected on the fly.
    for (int i = tid; i < DE; i += nth) {
      qvr[i] = 0.0;
      qvi[i] = 0.0;
      qwr[i] = 0.0;
      qwi[i] = 0.0;
    }
    __syncthreads();
    // pending correction of element (r, cc): v_r conj(w_cc) + w_r conj(v_cc)
    auto pend = [&](int r, int cc, double& ur, double& ui) {
      ur = fma(qvr[r], qwr[cc], fma(qvi[r], qwi[cc], fma(qwr[r], qvr[cc], qwi[r] * qvi[cc])));
      ui = fma(qvi[r], qwr[cc], fma(-qvr[r], qwi[cc], fma(qwi[r], qvr[cc], -qwr[r] * qvi[cc])));
    };
    for (int k = 0; k < DE - 2; ++k) {
      const int m = DE - k - 1;
      const int64_t rk = (int64_t)k * DE + k + 1;   // x_i = A[k+1+i][k] = conj(A[k][k+1+i])
      double xs = 0.0;
      for (int i = tid; i < m; i += nth) {
        double ur, ui;
        pend(k, k + 1 + i, ur, ui);
        const double xr = ar[rk + i] - ur;
        const double xim = CPLX ? ai[rk + i] - ui : 0.0;
        vr[i] = xr;     // x, turned into v below
        vi[i] = -xim;
        xs = fma(xr, xr, xs);
        if constexpr (CPLX) xs = fma(xim, xim, xs);
      }
      const double xn2 = block_sum(xs, red);
      const double xn = sqrt(xn2);
      const double x0r = vr[0], x0i = vi[0];
      const double a0 = sqrt(fma(x0r, x0r, x0i * x0i));
      if (tid == 0) {
        double ur, ui;
        pend(k, k, ur, ui);
        dg[k] = ar[(int64_t)k * DE + k] - ur;
        e2[k] = xn2;
      }
      const double vn2 = 2.0 * (xn2 + a0 * xn);
      // an already reduced column (block-uniform) reflects nothing (v = 0) but still flushes the
      // pending update into the trailing matrix
      const bool act = vn2 > 0.0;
      const double ur0 = a0 > 0.0 ? x0r / a0 : 1.0, ui0 = a0 > 0.0 ? x0i / a0 : 0.0;
      const double tau = act ? 2.0 / vn2 : 0.0;
      __syncthreads();
      if (act) {
        if (tid == 0) {   // v = x - alpha e1, alpha = -(x0/|x0|) ||x||
          vr[0] = fma(ur0, xn, x0r);
          vi[0] = fma(ui0, xn, x0i);
        }
      } else {
        for (int i = tid; i < m; i += nth) {
          vr[i] = 0.0;
          vi[i] = 0.0;
        }
      }
      __syncthreads();
      // p = tau A22 v on the updated A22, written back as it is read; A22 is Hermitian, so row i
      // of A22 v reads column i (coalesced across i)
      for (int i = tid; i < m; i += nth) {
        const int cc = k + 1 + i;
        const double wcr = qwr[cc], wci = qwi[cc], vcr = qvr[cc], vci = qvi[cc];
        double* col_r = ar + (int64_t)(k + 1) * DE + cc;
        double* col_i = CPLX ? ai + (int64_t)(k + 1) * DE + cc : nullptr;
        double sr = 0.0, si = 0.0;
#pragma unroll 4
        for (int j = 0; j < m; ++j) {
          const int r = k + 1 + j;
          const double a_r = col_r[(int64_t)j * DE] -
                             fma(qvr[r], wcr, fma(qvi[r], wci, fma(qwr[r], vcr, qwi[r] * vci)));
          col_r[(int64_t)j * DE] = a_r;
          sr = fma(a_r, vr[j], sr);
          if constexpr (CPLX) {
            const double b_i = col_i[(int64_t)j * DE] -
                               fma(qvi[r], wcr, fma(-qvr[r], wci, fma(qwi[r], vcr, -qwr[r] * vci)));
            col_i[(int64_t)j * DE] = b_i;
            const double a_i = -b_i;   // Im A[cc][r]
            sr = fma(-a_i, vi[j], sr);
            si = fma(a_r, vi[j], fma(a_i, vr[j], si));
          }
        }
        pr[i] = tau * sr;
        pi[i] = tau * si;
      }
      __syncthreads();
      double ks = 0.0;
      for (int i = tid; i < m; i += nth) ks = fma(vr[i], pr[i], fma(vi[i], pi[i], ks));
      const double K = 0.5 * tau * block_sum(ks, red);
      // the update of this reflection, A22 -= v w^H + w v^H with w = p - K v, becomes pending
      for (int i = tid; i < m; i += nth) {
        qvr[k + 1 + i] = vr[i];
        qvi[k + 1 + i] = vi[i];
        qwr[k + 1 + i] = fma(-K, vr[i], pr[i]);
        qwi[k + 1 + i] = fma(-K, vi[i], pi[i]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      double ur, ui;
      pend(DE - 2, DE - 2, ur, ui);
      dg[DE - 2] = ar[(int64_t)(DE - 2) * DE + DE - 2] - ur;
      pend(DE - 1, DE - 1, ur, ui);
      dg[DE - 1] = ar[(int64_t)(DE - 1) * DE + DE - 1] - ur;
      pend(DE - 2, DE - 1, ur, ui);
      const double xr = ar[(int64_t)(DE - 2) * DE + DE - 1] - ur;
      const double xi = CPLX ? ai[(int64_t)(DE - 2) * DE + DE - 1] - ui : 0.0;
      e2[DE - 2] = fma(xr, xr, xi * xi);
      e2[DE - 1] = 0.0;
    }
    __syncthreads();
    // Gershgorin bracket (every thread, same order: identical values)
    double lo = INFINITY, hi = -INFINITY, emax = 0.0;
    for (int i = 0; i < DE; ++i) {
      const double r = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + sqrt(e2[i]);
      lo = fmin(lo, dg[i] - r);
      hi = fmax(hi, dg[i] + r);
      emax = fmax(emax, e2[i]);
    }
    const double pivmin = DBL_MIN * fmax(1.0, emax);
    const double span0 = fmax(hi - lo, DBL_MIN);
    lo -= 2.0 * DBL_EPSILON * fabs(lo) + span0 * DBL_EPSILON;
    hi += 2.0 * DBL_EPSILON * fabs(hi) + span0 * DBL_EPSILON;
    for (int round = 0; round < 12; ++round) {
      if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;   // a few ulps of lambda_min
      const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(nth + 1);
      int cnt = 0;
      double q = dg[0] - x;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = 1; i < DE; ++i) {
        q = (dg[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
      const double first = block_min(cnt > 0 ? (double)tid : (double)nth, red);
      const int t = (int)first;
      const double nlo = t == 0 ? lo : lo + (hi - lo) * (double)t / (double)(nth + 1);
      const double nhi = t == nth ? hi : lo + (hi - lo) * (double)(t + 1) / (double)(nth + 1);
      if (!(nhi - nlo < hi - lo)) break;
      lo = nlo;
      hi = nhi;
    }
    const int32_t gid = A.gid[c];
    if (tid == 0) {
      A.scal[gid] = lo;
      A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt(nrm2);
      if (!isfinite(lo) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
    }
    __syncthreads();
  }
}

template <bool CPLX, int DE>
__global__ __launch_bounds__(256) void k_cluster_tridiag(ClusterArgs<double> A, double* scratch, int64_t slab) {
  constexpr int64_t DD = (int64_t)DE * DE;
  __shared__ double red[8];
  const int tid = threadIdx.x, nth = blockDim.x;
  double* ar = scratch + (int64_t)blockIdx.x * slab;
  double* ai = CPLX ? ar + DD : nullptr;
  for (int64_t c = blockIdx.x; c < A.n; c += gridDim.x) {
    const double my_n2 = big_assemble<double, double, CPLX, false>(A, c, DE, ar, ai, (double*)nullptr,
                                                                    (double*)nullptr, 0.0, tid, nth);
    tridiag_lambda_min<CPLX, DE>(A, c, ar, ai, block_sum(my_n2, red));
  }
}

// ------------------------------------------------------------------------------------------
// lambda_min-only certification, De = 64, 128, 256 (one workgroup of 256 threads per cluster)
// ------------------------------------------------------------------------------------------
//
// Q_C needs lambda_min of every theta_e and nothing else (Sec. 4.2).  Lanczos from a seeded
// start vector builds the tridiagonal T_k of theta_e on the Krylov space; its smallest
// eigenvalue rho is, by interlacing, at least lambda_min and converges to it, typically long
// before k = De.  rho is certified from below by one Cholesky factorisation of
// S = theta_e - sigma I at sigma = rho - eta.  If the factorisation runs to completion in
// floating point, the computed factor R satisfies R^H R = S + dS with |dS| <= g |R^H| |R|
// (backward error of Cholesky: g = gamma_{De+1} for real and sqrt(2) gamma_{2De+4} for complex
// arithmetic), so R^H R is positive semidefinite and
//     lambda_min(theta_e) >= sigma - g || |R| ||_2^2 - u max_i |theta_ii - sigma|
//                         >= sigma - g || |R| ||_1 || |R| ||_inf - u max_i |theta_ii - sigma|,
// the last term for the rounding of the shift.  The bound returned is that right-hand side less
// a term for the rounding of the assembly of theta_e; it is handed over as lambda = rho and
// margin = rho - bound.  If a pivot is not positive (rho not yet converged, or the start vector
// blind to the lowest eigenvector), the cluster is certified by the tridiagonalisation path
// instead (counted in the fallback counter).
//
// Memory: theta_e (full, row-major) in the workgroup's slab; Lanczos vectors, T_k and one
// column-major panel of NB columns of the factor in LDS.  A matrix-vector product reads the
// slab once (column t of the Hermitian theta_e gives row t of theta_e q, coalesced across t);
// the right-looking blocked factorisation reads and writes the trailing lower triangle once per
// panel.

// Smallest eigenvalue of the symmetric tridiagonal (al[0..k-1], off-diagonal be[0..k-2]) by
// multisection on Sturm counts with every thread of the workgroup, from the bracket
// [Gershgorin lower end, min_i al_i]; the midpoint of the final bracket.
__device__ double ritz_min(const double* al, const double* be, int k, double* red) {
  const int tid = threadIdx.x, nth = blockDim.x;
  double lo = INFINITY, hi = INFINITY, emax = 0.0;
  for (int i = 0; i < k; ++i) {   // every thread, same order: identical values
    const double bl = i > 0 ? be[i - 1] : 0.0, br = i + 1 < k ? be[i] : 0.0;
    lo = fmin(lo, al[i] - fabs(bl) - fabs(br));
    hi = fmin(hi, al[i]);
    emax = fmax(emax, br * br);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  for (int round = 0; round < 12; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;
    const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(nth + 1);
    int cnt = 0;
    double q = al[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
    for (int i = 1; i < k; ++i) {
      q = (al[i] - x) - be[i - 1] * be[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    const int t = (int)block_min(cnt > 0 ? (double)tid : (double)nth, red);
    const double nlo = t == 0 ? lo : lo + (hi - lo) * (double)t / (double)(nth + 1);
    const double nhi = t == nth ? hi : lo + (hi - lo) * (double)(t + 1) / (double)(nth + 1);
    if (!(nhi - nlo < hi - lo)) break;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {   // a 32-bit integer finaliser
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <bool CPLX, int DE>
__global__ __launch_bounds__(1024) void k_certify_lanczos(ClusterArgs<double> A, double* scratch, int64_t slab) {
  constexpr int64_t DD = (int64_t)DE * DE;
  constexpr int NT = 1024;
  constexpr int NW = NT / 64;
  constexpr int H = DE / 2;                  // shift-diagonals 0 .. H of the half storage
  constexpr int G = NT / DE;                 // threads per row in the matrix-vector product
  constexpr int KMAX = DE < 192 ? DE : 192;  // Lanczos steps at most
  constexpr int NB = 16;                     // Cholesky panel width (one wave per panel column)
  __shared__ double qr[DE], qi[CPLX ? DE : 1];
  __shared__ double yr[G][DE], yi[CPLX ? G : 1][CPLX ? DE : 1];
  __shared__ double al[KMAX], be[KMAX];
  __shared__ double Pr[NB][DE], Pi[CPLX ? NB : 1][CPLX ? DE : 1];
  __shared__ double rsum[DE];
  __shared__ double csum[NB];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int t = tid % DE, g = tid / DE;
  const double u = 0.5 * DBL_EPSILON;
  const int NBITS = log2i(DE);
  double* ar = scratch + (int64_t)blockIdx.x * slab;
  double* ai = CPLX ? ar + DD : nullptr;
  // half storage for the Lanczos products: B[s][t] = theta[(t + s) mod De][t], s = 0 .. De/2
  double* br = ar;
  double* bi = CPLX ? ar + (int64_t)(H + 1) * DE : nullptr;
  for (int64_t c = blockIdx.x; c < A.n; c += gridDim.x) {
    const int32_t gid = A.gid[c];
    const int64_t ho = A.hoff[c];
    double my = 0.0;
    for (int idx = tid; idx < (H + 1) * DE; idx += NT) {
      const int sh = idx / DE, tt = idx % DE;
      double vr_, vi_;
      theta_elem<double, CPLX>(A, c, DE, NBITS, ho, (tt + sh) & (DE - 1), tt, 0.0, vr_, vi_);
      br[idx] = vr_;
      if constexpr (CPLX) bi[idx] = vi_;
      // every off-diagonal pair once, except on the last shift-diagonal (twice there)
      const double w = (sh == 0 || sh == H) ? 1.0 : 2.0;
      my = fma(w * vr_, vr_, my);
      if constexpr (CPLX) my = fma(w * vi_, vi_, my);
    }
    const double nf = sqrt(block_sum(my, red));
    // ---- Lanczos ----
    my = 0.0;
    if (tid < DE) {
      const uint32_t h0 = mix32((uint32_t)gid * 0x9e3779b9u ^ mix32(2u * (uint32_t)tid + 1u));
      qr[tid] = (double)h0 * 0x1p-32 - 0.5;
      my = qr[tid] * qr[tid];
      if constexpr (CPLX) {
        qi[tid] = (double)mix32(h0 + 0x632be5abu) * 0x1p-32 - 0.5;
        my = fma(qi[tid], qi[tid], my);
      }
    }
    const double q0 = 1.0 / sqrt(block_sum(my, red));
    if (tid < DE) {
      qr[tid] *= q0;
      if constexpr (CPLX) qi[tid] *= q0;
    }
    double ppr = 0.0, ppi = 0.0, bprev = 0.0;   // q_{k-1} (thread tid < De) and beta_{k-1}
    double rho = INFINITY, rho_old = INFINITY, dlast = INFINITY;
    __syncthreads();
    for (int k = 0; k < KMAX; ++k) {
      {
        // (theta q)_t = sum_s conj(B[s][t]) q_{t+s} + sum_{0<s<H} B[s][t-s] q_{t-s}; both reads of
        // shift-diagonal s are coalesced across t (the second is the first rotated by s).
        // Thread (g, t) takes the shift-diagonals s = g mod G.
        double sr = 0.0, si = 0.0;
#pragma unroll 2
        for (int sh = g; sh <= H; sh += G) {
          const double* rr = br + (int64_t)sh * DE;
          const int up = (t + sh) & (DE - 1), dn = (t - sh) & (DE - 1);
          const bool two = sh > 0 && sh < H;
          const double b_r = rr[t];
          const double c_r = two ? rr[dn] : 0.0;
          double b_i = 0.0, c_i = 0.0;
          if constexpr (CPLX) {
            const double* ri = bi + (int64_t)sh * DE;
            b_i = ri[t];
            c_i = two ? ri[dn] : 0.0;
          }
          const double xr = qr[up], yr_ = qr[dn];
          sr = fma(b_r, xr, sr);
          sr = fma(c_r, yr_, sr);
          if constexpr (CPLX) {
            const double xi = qi[up], yi_ = qi[dn];
            sr = fma(b_i, xi, sr);
            sr = fma(-c_i, yi_, sr);
            si = fma(b_r, xi, fma(-b_i, xr, si));
            si = fma(c_r, yi_, fma(c_i, yr_, si));
          }
        }
        yr[g][t] = sr;
        if constexpr (CPLX) yi[g][t] = si;
      }
      __syncthreads();
      double wr = 0.0, wi = 0.0, ma = 0.0;
      if (tid < DE) {
#pragma unroll
        for (int h = 0; h < G; ++h) {
          wr += yr[h][tid];
          if constexpr (CPLX) wi += yi[h][tid];
        }
        wr = fma(-bprev, ppr, wr);
        ma = qr[tid] * wr;
        if constexpr (CPLX) {
          wi = fma(-bprev, ppi, wi);
          ma = fma(qi[tid], wi, ma);
        }
      }
      const double alpha = block_sum(ma, red);
      double mb = 0.0;
      if (tid < DE) {
        wr = fma(-alpha, qr[tid], wr);
        mb = wr * wr;
        if constexpr (CPLX) {
          wi = fma(-alpha, qi[tid], wi);
          mb = fma(wi, wi, mb);
        }
      }
      const double beta = sqrt(block_sum(mb, red));
      const bool invariant = !(beta > 64.0 * u * nf);   // Krylov space invariant (or no progress)
      if (tid == 0) {
        al[k] = alpha;
        be[k] = beta;
      }
      if (tid < DE) {
        ppr = qr[tid];
        if constexpr (CPLX) ppi = qi[tid];
        if (!invariant) {
          const double ib = 1.0 / beta;
          qr[tid] = wr * ib;
          if constexpr (CPLX) qi[tid] = wi * ib;
        }
      }
      bprev = beta;
      __syncthreads();
      const int kk = k + 1;
      if (invariant || kk == KMAX || (kk >= 16 && (kk & 7) == 0)) {
        rho = ritz_min(al, be, kk, red);
        dlast = invariant ? 0.0 : fabs(rho_old - rho);
        rho_old = rho;
        if (dlast <= 64.0 * u * nf) break;
      }
    }
    // the full matrix for the factorisation, over the half storage
    big_assemble<double, double, CPLX, false>(A, c, DE, ar, ai, (double*)nullptr, (double*)nullptr, 0.0, tid, NT);
    __syncthreads();
    // ---- Cholesky of theta - sigma I, sigma = rho - eta ----
    const double eta = 2.0 * dlast + 16.0 * DE * u * nf;
    const double sigma = A.cert_method == 2 ? rho + 1.0 + nf : rho - eta;
    bool ok = isfinite(sigma) && dlast <= 1e-10 * nf;   // unconverged Ritz value: fall back
    double dmax = 0.0, cmax = 0.0;
    for (int i = tid; i < DE; i += NT) rsum[i] = 0.0;
    for (int p = 0; p < DE && ok; p += NB) {
      const int m = DE - p;   // rows p .. De-1 of the panel
      for (int idx = tid; idx < m * NB; idx += NT) {
        const int r = idx / NB, q = idx % NB;
        const int64_t o = (int64_t)(p + r) * DE + p + q;
        double vr_ = ar[o], vi_ = CPLX ? ai[o] : 0.0;
        if (r == q) {
          vr_ -= sigma;
          vi_ = 0.0;
          dmax = fmax(dmax, fabs(vr_));
        }
        Pr[q][r] = vr_;
        if constexpr (CPLX) Pi[q][r] = vi_;
      }
      __syncthreads();
      for (int q = 0; q < NB; ++q) {
        const double d = Pr[q][q];
        if (!(d > 0.0) || !isfinite(d)) {   // every thread reads the same value: uniform
          ok = false;
          break;
        }
        const double l = sqrt(d), il = 1.0 / l;
        __syncthreads();
        for (int r = q + tid; r < m; r += NT) {
          Pr[q][r] = r == q ? l : Pr[q][r] * il;
          if constexpr (CPLX) Pi[q][r] = r == q ? 0.0 : Pi[q][r] * il;
        }
        __syncthreads();
        // S[r][q2] -= L[r][q] conj(L[q2][q]) for the panel's later columns q2 <= r (wave per column)
        for (int q2 = q + 1 + wave; q2 < NB; q2 += NW) {
          const double kr = Pr[q][q2], ki = CPLX ? Pi[q][q2] : 0.0;
          for (int r = q2 + lane; r < m; r += 64) {
            const double lr = Pr[q][r];
            if constexpr (CPLX) {
              const double li = Pi[q][r];
              Pr[q2][r] -= fma(lr, kr, li * ki);
              Pi[q2][r] -= fma(li, kr, -lr * ki);
            } else {
              Pr[q2][r] -= lr * kr;
            }
          }
        }
        __syncthreads();
      }
      if (!ok) break;
      // sums of |L| along the panel's rows (this thread's rows) and columns (wave per column)
      for (int r = tid; r < m; r += NT) {
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (r < q) continue;
          rs += CPLX ? sqrt(fma(Pr[q][r], Pr[q][r], Pi[q][r] * Pi[q][r])) : fabs(Pr[q][r]);
        }
        rsum[p + r] += rs;
      }
      for (int q = wave; q < NB; q += NW) {
        double cs = 0.0;
        for (int r = q + lane; r < m; r += 64)
          cs += CPLX ? sqrt(fma(Pr[q][r], Pr[q][r], Pi[q][r] * Pi[q][r])) : fabs(Pr[q][r]);
        cs = wave_sum(cs);
        if (lane == 0) csum[q] = cs;
      }
      // trailing update S[i][j] -= sum_q L[i][q] conj(L[j][q]), i >= j >= p + NB: wave per row
      const int mt = m - NB;
      for (int r = wave; r < mt; r += NW) {
        const int i = NB + r;
        for (int cc = lane; cc <= r; cc += 64) {
          const int j = NB + cc;
          double sr = 0.0, si = 0.0;
#pragma unroll 4
          for (int q = 0; q < NB; ++q) {
            const double ar_ = Pr[q][i], br_ = Pr[q][j];
            sr = fma(ar_, br_, sr);
            if constexpr (CPLX) {
              const double ai_ = Pi[q][i], bi_ = Pi[q][j];
              sr = fma(ai_, bi_, sr);
              si = fma(ai_, br_, fma(-ar_, bi_, si));
            }
          }
          const int64_t o = (int64_t)(p + i) * DE + p + j;
          ar[o] -= sr;
          if constexpr (CPLX) ai[o] -= si;
        }
      }
      __syncthreads();
      if (tid == 0)
        for (int q = 0; q < NB; ++q) cmax = fmax(cmax, csum[q]);
    }
    ok = ok && A.cert_method != 2;
    if (ok) {
      double rmax = 0.0;
      for (int i = tid; i < DE; i += NT) rmax = fmax(rmax, rsum[i]);
      rmax = block_max(rmax, red);
      dmax = block_max(dmax, red);
      if (tid == 0) {
        constexpr double nn = CPLX ? 2.0 * DE + 4.0 : DE + 1.0;
        const double gam = (CPLX ? 1.4142135623730951 : 1.0) * nn * u / (1.0 - nn * u);
        const double c_chol = gam * cmax * rmax * (1.0 + 4.0 * DE * u);
        const double c_shift = 2.0 * u * dmax;
        const double c_asm = 2.0 * (A.maxch + A.maxpar + 1) * u * nf;
        A.scal[gid] = rho;
        A.scal2[gid] = (rho - sigma) + c_chol + c_shift + c_asm;
        if (!isfinite(rho) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
      }
      __syncthreads();
    } else {
      if (tid == 0 && A.cert_fallback) atomicAdd(A.cert_fallback, 1ull);
      const double n2 = block_sum(big_assemble<double, double, CPLX, false>(A, c, DE, ar, ai, (double*)nullptr,
                                                                            (double*)nullptr, 0.0, tid, NT), red);
      tridiag_lambda_min<CPLX, DE>(A, c, ar, ai, n2);
    }
  }
}

// Bits of a placed, lowest first, at the set bits of mask (lowest first).
__device__ __forceinline__ int spread_bits(int a, int mask) {
  int r = 0;
  for (int t = 0; mask != 0; ++t) {
    const int lb = mask & -mask;
    if ((a >> t) & 1) r |= lb;
    mask ^= lb;
  }
  return r;
}

// theta_e at the messages (no extrapolation) into the group's LDS matrix, De lanes per cluster
// (lane i): h_e and the parent messages row by row, then the child messages entry by entry, each
// entry (a, b) of 1 (x) nu_{e->f} scattered to its De / Dc positions (pdep(a, x), pdep(b, x)) over
// the complement bits x.  Children go one after another: two of them can reach one element.
template <bool CPLX, int DE>
__device__ void rows_assemble(const ClusterArgs<double>& A, int64_t c, int i, bool active, double* dr, double* di) {
  constexpr int LD = DE + 1;
  double rr[DE], ri[CPLX ? DE : 1];
#pragma unroll
  for (int j = 0; j < DE; ++j) {
    rr[j] = 0.0;
    if constexpr (CPLX) ri[j] = 0.0;
  }
  const int64_t ho = active ? A.hoff[c] : -1;
  if (ho >= 0) {
    const double* h = A.h + ho;
#pragma unroll
    for (int j = 0; j < DE; ++j) {
      double vr, vi;
      herm_elem<double>([&](int k) { return h[k]; }, i, j, DE, CPLX, vr, vi);
      rr[j] = vr;
      if constexpr (CPLX) ri[j] = vi;
    }
  }
  for (int s = 0; s < A.maxpar; ++s) {
    const int m = active ? A.par[(int64_t)s * A.n + c] : -1;
    if (m < 0) continue;
#pragma unroll
    for (int j = 0; j < DE; ++j) {
      double vr, vi;
      herm_elem<double>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, i, j, DE, CPLX, vr, vi);
      rr[j] += vr;
      if constexpr (CPLX) ri[j] += vi;
    }
  }
#pragma unroll
  for (int j = 0; j < DE; ++j) {
    dr[i * LD + j] = rr[j];
    if constexpr (CPLX) di[i * LD + j] = ri[j];
  }
  __syncthreads();
  if (A.Dc <= 0) return;
  const int Dc = A.Dc, ldc = __builtin_ctz(Dc), NE = Dc * Dc;
  for (int s = 0; s < A.maxch; ++s) {   // maxch is the bucket's: the barrier below is uniform
    const int m = active ? A.ch[(int64_t)s * A.n + c] : -1;
    if (m >= 0) {
      const int mask = A.chmask[(int64_t)s * A.n + c] & (DE - 1);
      const int cm = ~mask & (DE - 1);
      for (int ab = i; ab < NE; ab += DE) {
        const int a = ab >> ldc, b = ab & (Dc - 1);
        double er, ei;
        herm_elem<double>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, a, b, Dc, CPLX, er, ei);
        const int ia = spread_bits(a, mask), jb = spread_bits(b, mask);
        int x = 0;
        do {   // every subset x of the complement bits
          dr[(ia | x) * LD + (jb | x)] -= er;
          if constexpr (CPLX) di[(ia | x) * LD + (jb | x)] -= ei;
          x = (x - cm) & cm;
        } while (x != 0);
      }
    }
    __syncthreads();
  }
}

// Row-parallel variant for De = 16, 32 (the default there): De lanes per cluster, 64 / De
// clusters per wave, lane i holding row i of theta_e in registers.  Column k below the diagonal
// is then one register per lane, the vectors v and w of each reflection are exchanged through
// LDS, and the reductions stay inside the lane group.  The tridiagonal (d, |e|^2) goes to a
// workspace (structure of arrays: d_k of cluster c at ws[k n + c], |e_k|^2 at ws[(De + k) n + c])
// for k_sturm_bisect, which brackets lambda_min with one lane per cluster.
template <bool CPLX, int DE>
__global__ __launch_bounds__(64) void k_certify_rows(ClusterArgs<double> A, double* ws) {
  constexpr int LD = DE + 1;
  constexpr int G = 64 / DE;
  __shared__ double sar[G * DE * LD];
  __shared__ double sai[CPLX ? G * DE * LD : 1];
  __shared__ double vbr[G][DE], vbi[G][CPLX ? DE : 1], wbr[G][DE], wbi[G][CPLX ? DE : 1];
  const int l = threadIdx.x, g = l / DE, i = l % DE;
  const int64_t c = (int64_t)blockIdx.x * G + g;
  const bool active = c < A.n;
  double* dr = sar + g * DE * LD;
  double* di = CPLX ? sai + g * DE * LD : sai;
  rows_assemble<CPLX, DE>(A, c, i, active, dr, di);
  double ar[DE], ai[CPLX ? DE : 1];
  double n2 = 0.0;
#pragma unroll
  for (int j = 0; j < DE; ++j) {
    ar[j] = active ? dr[i * LD + j] : 0.0;
    n2 = fma(ar[j], ar[j], n2);
    if constexpr (CPLX) {
      ai[j] = active ? di[i * LD + j] : 0.0;
      n2 = fma(ai[j], ai[j], n2);
    }
  }
  const double nrm2 = seg_sum<DE>(n2);
  double e2mine = 0.0;
#pragma unroll
  for (int k = 0; k < DE - 2; ++k) {
    // x = column k below the diagonal: element k of the rows i > k
    const bool below = i > k;
    const double xr = below ? ar[k] : 0.0;
    const double xi = (CPLX && below) ? ai[k] : 0.0;
    const double xn2 = seg_sum<DE>(fma(xr, xr, xi * xi));
    if (i == k) e2mine = xn2;
    // x0 = element k + 1, the first of x, broadcast from lane k + 1 of the group
    const double x0r = __shfl(xr, g * DE + k + 1, 64), x0i = CPLX ? __shfl(xi, g * DE + k + 1, 64) : 0.0;
    const double xn = sqrt(xn2), a0 = sqrt(fma(x0r, x0r, x0i * x0i));
    const double vn2 = 2.0 * (xn2 + a0 * xn);
    const bool act = vn2 > 0.0;      // uniform in the group: nothing to reflect when x = 0
    const double tau = act ? 2.0 / vn2 : 0.0;
    const double ur = a0 > 0.0 ? x0r / a0 : 1.0, ui = a0 > 0.0 ? x0i / a0 : 0.0;
    // v = x - alpha e_{k+1}, alpha = -(x0 / |x0|) ||x||
    double vr = xr, vi = xi;
    if (i == k + 1) {
      vr = fma(ur, xn, vr);
      vi = fma(ui, xn, vi);
    }
    vbr[g][i] = vr;
    if constexpr (CPLX) vbi[g][i] = vi;
    __syncthreads();
    // p_i = tau sum_{j > k} A_ij v_j
    double pr = 0.0, pim = 0.0;
#pragma unroll
    for (int j = k + 1; j < DE; ++j) {
      const double bjr = vbr[g][j];
      pr = fma(ar[j], bjr, pr);
      if constexpr (CPLX) {
        const double bji = vbi[g][j];
        pr = fma(-ai[j], bji, pr);
        pim = fma(ar[j], bji, fma(ai[j], bjr, pim));
      }
    }
    pr *= tau;
    pim *= tau;
    // K = (tau / 2) v^H p (real), w = p - K v
    const double K = 0.5 * tau * seg_sum<DE>(fma(vr, pr, vi * pim));
    const double wr = fma(-K, vr, pr), wi = fma(-K, vi, pim);
    wbr[g][i] = wr;
    if constexpr (CPLX) wbi[g][i] = wi;
    __syncthreads();
    // A22 -= v w^H + w v^H (lanes i <= k have v_i = w_i = 0: their rows do not change)
#pragma unroll
    for (int j = k + 1; j < DE; ++j) {
      const double vjr = vbr[g][j], wjr = wbr[g][j];
      if constexpr (CPLX) {
        const double vji = vbi[g][j], wji = wbi[g][j];
        ar[j] -= fma(vr, wjr, fma(vi, wji, fma(wr, vjr, wi * vji)));
        ai[j] -= fma(vi, wjr, fma(-vr, wji, fma(wi, vjr, -wr * vji)));
      } else {
        ar[j] -= fma(vr, wjr, wr * vjr);
      }
    }
    __syncthreads();   // before the next step overwrites the broadcast vectors
  }
  // last 2 x 2 block: |e_{De-2}|^2 = |A_{De-2, De-1}|^2, element De - 1 of row De - 2
  if (i == DE - 2) e2mine = fma(ar[DE - 1], ar[DE - 1], CPLX ? ai[DE - 1] * ai[DE - 1] : 0.0);
  double dmine = 0.0;
#pragma unroll
  for (int j = 0; j < DE; ++j)
    if (j == i) dmine = ar[j];
  if (active) {
    ws[(int64_t)i * A.n + c] = dmine;
    ws[(int64_t)(DE + i) * A.n + c] = (i < DE - 1) ? e2mine : 0.0;
    if (i == 0) A.scal2[A.gid[c]] = 8.0 * DE * DBL_EPSILON * sqrt(nrm2);
  }
}

// lambda_min of every cluster's tridiagonal (d, |e|^2) by bisection on Sturm counts, one lane per
// cluster: from the Gershgorin interval (widened by a few ulps) down to a few ulps of lambda_min;
// the lower end of the final bracket, below which the tridiagonal has no eigenvalue, is returned.
template <int DE>
__global__ __launch_bounds__(256) void k_sturm_bisect(ClusterArgs<double> A, const double* ws) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= A.n) return;
  double d[DE], e2[DE];
#pragma unroll
  for (int k = 0; k < DE; ++k) {
    d[k] = ws[(int64_t)k * A.n + c];
    e2[k] = ws[(int64_t)(DE + k) * A.n + c];
  }
  double lo = INFINITY, hi = -INFINITY, emax = 0.0, re_prev = 0.0;
#pragma unroll
  for (int k = 0; k < DE; ++k) {
    const double re = sqrt(e2[k]);
    lo = fmin(lo, d[k] - (re_prev + re));
    hi = fmax(hi, d[k] + (re_prev + re));
    emax = fmax(emax, e2[k]);
    re_prev = re;
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double span0 = fmax(hi - lo, DBL_MIN);
  lo -= 2.0 * DBL_EPSILON * fabs(lo) + span0 * DBL_EPSILON;
  hi += 2.0 * DBL_EPSILON * fabs(hi) + span0 * DBL_EPSILON;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;
    const double x = 0.5 * (lo + hi);
    if (!(x > lo && x < hi)) break;
    bool neg = false;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    neg = q < 0.0;
#pragma unroll
    for (int k = 1; k < DE; ++k) {
      q = (d[k] - x) - e2[k - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      neg = neg || (q < 0.0);
    }
    if (neg) hi = x;   // an eigenvalue below x
    else lo = x;
  }
  const int32_t gid = A.gid[c];
  A.scal[gid] = lo;
  if (!isfinite(lo) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
}

// One-wave variant for De = 16, 32: the matrix in LDS, the De rows of A22 v split over
// 64/De lane groups (partial sums over j = g, g + G, ... combined by shuffles), 64 Sturm
// points per multisection round.
template <bool CPLX, int DE>
__global__ __launch_bounds__(64) void k_cluster_tridiag_w(ClusterArgs<double> A) {
  constexpr int LD = DE + 1;
  constexpr int G = 64 / DE;
  __shared__ double ar[DE * LD];
  __shared__ double ai[CPLX ? DE * LD : 1];
  __shared__ double vr[DE], vi[DE], pr[DE], pi[DE], dg[DE], e2[DE];
  const int64_t c = xcd_cluster(blockIdx.x, A.n);
  const int l = threadIdx.x;
  const int li = l % DE, lg = l / DE;
  const double nrm2 = wave_sum_dpp(
      lds_assemble<double, CPLX, DE, 64>(A, c, l, A.nu_c, nullptr, A.nu_p, nullptr, 0.0, true, 1.0, ar, ai));
  __syncthreads();
  for (int k = 0; k < DE - 2; ++k) {
    const int m = DE - k - 1;
    const int rk = k * LD + k + 1;   // x_i = A[k+1+i][k] = conj(A[k][k+1+i])
    double xs = 0.0;
    if (l < m) {
      xs = ar[rk + l] * ar[rk + l];
      if constexpr (CPLX) xs = fma(ai[rk + l], ai[rk + l], xs);
    }
    const double xn2 = wave_sum_dpp(xs);
    const double xn = sqrt(xn2);
    const double x0r = ar[rk], x0i = CPLX ? -ai[rk] : 0.0;
    const double a0 = sqrt(fma(x0r, x0r, x0i * x0i));
    if (l == 0) {
      dg[k] = ar[k * LD + k];
      e2[k] = xn2;
    }
    const double vn2 = 2.0 * (xn2 + a0 * xn);
    if (!(vn2 > 0.0)) continue;   // wave-uniform
    const double ur = a0 > 0.0 ? x0r / a0 : 1.0, ui = a0 > 0.0 ? x0i / a0 : 0.0;
    const double tau = 2.0 / vn2;
    if (l < m) {
      double r = ar[rk + l], im = CPLX ? -ai[rk + l] : 0.0;
      if (l == 0) {
        r += ur * xn;
        im += ui * xn;
      }
      vr[l] = r;
      vi[l] = im;
    }
    __syncthreads();
    // p = tau A22 v: lane (li, lg) sums j = lg, lg + G, ... of row li (read as column li)
    double sr = 0.0, si = 0.0;
    if (li < m) {
      for (int j = lg; j < m; j += G) {
        const int o = (k + 1 + j) * LD + (k + 1 + li);
        const double a_r = ar[o];
        sr = fma(a_r, vr[j], sr);
        if constexpr (CPLX) {
          const double a_i = -ai[o];
          sr = fma(-a_i, vi[j], sr);
          si = fma(a_r, vi[j], fma(a_i, vr[j], si));
        }
      }
    }
#pragma unroll
    for (int o = DE; o < 64; o <<= 1) {
      sr += __shfl_xor(sr, o, 64);
      if constexpr (CPLX) si += __shfl_xor(si, o, 64);
    }
    sr *= tau;
    si *= tau;
    const double ks = (l < m) ? fma(vr[l], sr, vi[l] * si) : 0.0;
    const double K = 0.5 * tau * wave_sum_dpp(ks);
    if (l < m) {
      pr[l] = fma(-K, vr[l], sr);
      pi[l] = fma(-K, vi[l], si);
    }
    __syncthreads();
    // A22 -= v w^H + w v^H: lane (li, lg) updates column li of rows lg, lg + G, ... (no division)
    if (li < m) {
#pragma unroll 4
      for (int i = lg; i < m; i += G) {
        const int o = (k + 1 + i) * LD + (k + 1 + li);
        ar[o] -= fma(vr[i], pr[li], fma(vi[i], pi[li], fma(pr[i], vr[li], pi[i] * vi[li])));
        if constexpr (CPLX) ai[o] -= fma(vi[i], pr[li], fma(-vr[i], pi[li], fma(pi[i], vr[li], -pr[i] * vi[li])));
      }
    }
    __syncthreads();
  }
  if (l == 0) {
    dg[DE - 2] = ar[(DE - 2) * LD + DE - 2];
    dg[DE - 1] = ar[(DE - 1) * LD + DE - 1];
    const double xr = ar[(DE - 2) * LD + DE - 1], xi = CPLX ? ai[(DE - 2) * LD + DE - 1] : 0.0;
    e2[DE - 2] = fma(xr, xr, xi * xi);
    e2[DE - 1] = 0.0;
  }
  __syncthreads();
  double lo = INFINITY, hi = -INFINITY, emax = 0.0;
  for (int i = 0; i < DE; ++i) {
    const double r = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + sqrt(e2[i]);
    lo = fmin(lo, dg[i] - r);
    hi = fmax(hi, dg[i] + r);
    emax = fmax(emax, e2[i]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double span0 = fmax(hi - lo, DBL_MIN);
  lo -= 2.0 * DBL_EPSILON * fabs(lo) + span0 * DBL_EPSILON;
  hi += 2.0 * DBL_EPSILON * fabs(hi) + span0 * DBL_EPSILON;
  for (int round = 0; round < 14; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;   // a few ulps of lambda_min
    const double x = lo + (hi - lo) * (double)(l + 1) / 65.0;
    int cnt = 0;
    double q = dg[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
    for (int i = 1; i < DE; ++i) {
      q = (dg[i] - x) - e2[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    const int t = (int)wave_min_dpp(cnt > 0 ? (double)l : 64.0);
    const double nlo = t == 0 ? lo : lo + (hi - lo) * (double)t / 65.0;
    const double nhi = t == 64 ? hi : lo + (hi - lo) * (double)(t + 1) / 65.0;
    if (!(nhi - nlo < hi - lo)) break;
    lo = nlo;
    hi = nhi;
  }
  const int32_t gid = A.gid[c];
  if (l == 0) {
    A.scal[gid] = lo;
    A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt(nrm2);
    if (!isfinite(lo) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  }
}

// ------------------------------------------------------------------------------------------
// adjoint (a9): VJP of (Q_beta, grad Q_beta) through one cluster
// ------------------------------------------------------------------------------------------
//
// grad Q_beta = B^* rho_beta(B nu + h) with B the linear map from messages to augmented
// Hamiltonians (chain rule of the Lipschitz lemma, Sec. 4.1.2).  For cotangents qbar (per
// instance) and gbar (per message) the cluster's cotangent is
//     Y_e = qbar rho_e + D rho_e[(B gbar)_e],
// with the Daleckii-Krein derivative of the normalised matrix exponential
//     D rho[X] = U [Gamma o (U^H X U)] U^H + beta <rho, X> rho,
//     Gamma_ab = (p_a - p_b)/(l_a - l_b) = p_lo expm1(-beta (l_hi - l_lo)) / (l_hi - l_lo),
//     Gamma_aa = -beta p_a.
// nu_bar = B^* Y is then the message kernel's gradient stage (Y_f - Tr_{e\f} Y_e).  At beta = 0
// the cotangent of Q is Y_e = qbar mu_e (the ground projector; gbar must be absent).
template <typename T, bool CPLX, int DE, int MODE>
__global__ __launch_bounds__(64) void k_cluster_vjp(ClusterArgs<T> A) {
  constexpr int LD = DE + 1;
  __shared__ T sar[DE * LD];
  __shared__ T sai[CPLX ? DE * LD : 1];
  __shared__ T sur[DE * LD];
  __shared__ T sui[CPLX ? DE * LD : 1];
  __shared__ T sxr[DE * LD];
  __shared__ T sxi[CPLX ? DE * LD : 1];
  __shared__ T str[DE * LD];
  __shared__ T sti[CPLX ? DE * LD : 1];
  __shared__ JacobiScratch<T, DE / 2> J;
  __shared__ T sp[DE];
  __shared__ T slam[DE];
  const int64_t c = xcd_cluster(blockIdx.x, A.n);
  if (c >= A.n) return;
  const int tid = threadIdx.x;
  const bool has_g = (A.gb_c != nullptr || A.gb_p != nullptr);
  const T nrm2 = wave_sum(lds_assemble<T, CPLX, DE, 64>(A, c, tid, A.nu_c, nullptr, A.nu_p, nullptr, T(0), true,
                                                        T(1), sar, sai));
  if (has_g) lds_assemble<T, CPLX, DE, 64>(A, c, tid, A.gb_c, nullptr, A.gb_p, nullptr, T(0), false,
                                           (T)A.gb_offscale, sxr, sxi);
  for (int idx = tid; idx < DE * DE; idx += 64) {
    const int i = idx / DE, j = idx % DE;
    sur[i * LD + j] = (i == j) ? T(1) : T(0);
    if constexpr (CPLX) sui[i * LD + j] = T(0);
  }
  __syncthreads();
  const bool conv = lds_jacobi<T, CPLX, DE, true, 64>(sar, sai, sur, sui, J, A.tol * A.tol * (double)nrm2,
                                                      A.max_sweeps, tid, true);
  if (!conv && tid == 0 && A.noconv) atomicAdd(A.noconv, 1ull);
  T lmin = T(INFINITY);
  for (int k = tid; k < DE; k += 64) {
    slam[k] = sar[k * LD + k];
    lmin = fmin(lmin, sar[k * LD + k]);
  }
  lmin = wave_min(lmin);
  const T beta = (T)A.beta;
  lds_weights<T, DE, MODE, 64>(sar, sp, lmin, beta, (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2)), tid, true);
  // rho (or mu) over A
  lds_rebuild<T, CPLX, DE, 64>(sur, sui, sp, sar, sai, tid);
  __syncthreads();
  const int32_t gid = A.gid[c];
  const T qb = A.qbar ? (T)A.qbar[A.cinst[gid]] : T(0);
  if (MODE == MODE_GIBBS && has_g) {
    // <rho, X>
    T rx = T(0);
    for (int idx = tid; idx < DE * DE; idx += 64) {
      rx = dfma<T>(sar[idx / DE * LD + idx % DE], sxr[idx / DE * LD + idx % DE], rx);
      if constexpr (CPLX) rx = dfma<T>(sai[idx / DE * LD + idx % DE], sxi[idx / DE * LD + idx % DE], rx);
    }
    rx = wave_sum(rx);
    // Tm = U^H X
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int a = idx / DE, j = idx % DE;
      T sr = T(0), si = T(0);
      for (int k = 0; k < DE; ++k) {
        const T ur = sur[k * LD + a], ui = CPLX ? -sui[k * LD + a] : T(0);  // conj(U_ka)
        const T xr = sxr[k * LD + j], xi = CPLX ? sxi[k * LD + j] : T(0);
        sr = dfma<T>(ur, xr, sr);
        if constexpr (CPLX) {
          sr = dfma<T>(-ui, xi, sr);
          si = dfma<T>(ur, xi, si);
          si = dfma<T>(ui, xr, si);
        }
      }
      str[a * LD + j] = sr;
      if constexpr (CPLX) sti[a * LD + j] = si;
    }
    __syncthreads();
    // M = (U^H X) U, then Gamma o M (into X)
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int a = idx / DE, b = idx % DE;
      T sr = T(0), si = T(0);
      for (int k = 0; k < DE; ++k) {
        const T tr = str[a * LD + k], ti = CPLX ? sti[a * LD + k] : T(0);
        const T ur = sur[k * LD + b], ui = CPLX ? sui[k * LD + b] : T(0);
        sr = dfma<T>(tr, ur, sr);
        if constexpr (CPLX) {
          sr = dfma<T>(-ti, ui, sr);
          si = dfma<T>(tr, ui, si);
          si = dfma<T>(ti, ur, si);
        }
      }
      const int hi = slam[a] >= slam[b] ? a : b, lo = slam[a] >= slam[b] ? b : a;
      const T dl = slam[hi] - slam[lo];
      const T g = (dl == T(0)) ? -beta * sp[lo] : sp[lo] * (T)expm1((double)(-beta * dl)) / dl;
      sxr[a * LD + b] = g * sr;
      if constexpr (CPLX) sxi[a * LD + b] = g * si;
    }
    __syncthreads();
    // Tm = U (Gamma o M)
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int i = idx / DE, b = idx % DE;
      T sr = T(0), si = T(0);
      for (int k = 0; k < DE; ++k) {
        const T ur = sur[i * LD + k], ui = CPLX ? sui[i * LD + k] : T(0);
        const T mr = sxr[k * LD + b], mi = CPLX ? sxi[k * LD + b] : T(0);
        sr = dfma<T>(ur, mr, sr);
        if constexpr (CPLX) {
          sr = dfma<T>(-ui, mi, sr);
          si = dfma<T>(ur, mi, si);
          si = dfma<T>(ui, mr, si);
        }
      }
      str[i * LD + b] = sr;
      if constexpr (CPLX) sti[i * LD + b] = si;
    }
    __syncthreads();
    // Y = Tm U^H + (beta <rho,X> + qbar) rho  (into X)
    const T w = beta * rx + qb;
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int i = idx / DE, j = idx % DE;
      T sr = T(0), si = T(0);
      for (int k = 0; k < DE; ++k) {
        const T tr = str[i * LD + k], ti = CPLX ? sti[i * LD + k] : T(0);
        const T ur = sur[j * LD + k], ui = CPLX ? -sui[j * LD + k] : T(0);  // conj(U_jk)
        sr = dfma<T>(tr, ur, sr);
        if constexpr (CPLX) {
          sr = dfma<T>(-ti, ui, sr);
          si = dfma<T>(tr, ui, si);
          si = dfma<T>(ti, ur, si);
        }
      }
      sxr[i * LD + j] = dfma<T>(w, sar[i * LD + j], sr);
      if constexpr (CPLX) sxi[i * LD + j] = dfma<T>(w, sai[i * LD + j], si);
    }
    __syncthreads();
    // symmetrise (Y is Hermitian up to rounding): keep the upper triangle mirrored
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int i = idx / DE, j = idx % DE;
      if (i < j) {
        sxr[j * LD + i] = sxr[i * LD + j];
        if constexpr (CPLX) sxi[j * LD + i] = -sxi[i * LD + j];
      }
      if constexpr (CPLX) { if (i == j) sxi[i * LD + i] = T(0); }
    }
    __syncthreads();
    lds_outputs<T, CPLX, DE, 64>(A, c, tid, gid, sxr, sxi);
  } else {
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int i = idx / DE, j = idx % DE;
      sxr[i * LD + j] = qb * sar[i * LD + j];
      if constexpr (CPLX) sxi[i * LD + j] = qb * sai[i * LD + j];
    }
    __syncthreads();
    lds_outputs<T, CPLX, DE, 64>(A, c, tid, gid, sxr, sxi);
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Register (one lane per cluster) instantiations: which (De, precision, field, mode) fit the
// register file (the whole De x De matrix and, with vectors, U live in one lane's VGPRs).
template <typename T, bool CPLX, int DE, int MODE>
constexpr bool reg_ok() {
  constexpr bool dbl = std::is_same<T, double>::value;
  if constexpr (DE <= 4) return true;
  if constexpr (DE == 8) return !(dbl && CPLX && MODE != MODE_CERTIFY);
  return false;  // D_e = 16: H + U exceed the arch VGPR file of one lane; the LDS kernel takes it
}

// Scaling-and-squaring Gibbs kernel (shape code W = 0): dimensions and fields compiled.
static bool expm_ok(int De, bool cplx) { return De == 16 || De == 32 || De == 64 || De == 128 || De == 256; }

// (childless 4 x 4 and 8 x 8 clusters are the overlaps of the two-level family)
static bool reg_pair(int De, int Dc) {
  return (De == 2 && Dc == 0) || (De == 4 && (Dc == 2 || Dc == 0)) || (De == 8 && (Dc == 4 || Dc == 2 || Dc == 0));
}

template <typename T, bool CPLX, int MODE, int DE, int W>
static void launch_lds_w(const ClusterArgs<T>& a, hipStream_t s) {
  constexpr int G = 64 / W;
  hipLaunchKernelGGL((k_cluster_lds<T, CPLX, DE, MODE, W>), dim3((unsigned)((a.n + G - 1) / G)), dim3(64), 0, s, a);
}

template <typename T, bool CPLX, int MODE, int DE, int DC>
static hipError_t launch_reg(const ClusterArgs<T>& a, int block, hipStream_t s) {
  if constexpr (reg_ok<T, CPLX, DE, MODE>()) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, DE, DC, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, bool CPLX, int MODE>
static hipError_t launch_cluster_m(const ClusterArgs<T>& a, int block, int W, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  // the register kernels hold one slot per site for single-site children
  if (a.Dc == 2 && (a.maxch < 1 || a.maxch > log2i(a.De))) return hipErrorInvalidValue;
  if (a.Dc == 2 && a.fp != nullptr && a.ch_rslot == nullptr) return hipErrorInvalidValue;
  if (W == 0 || W == 4) {   // 0: one wave per cluster up to D = 32, 4: one workgroup per cluster
    if constexpr (MODE == MODE_GIBBS) {
      if (a.fp != nullptr || a.n > 0x7fffffff) return hipErrorInvalidValue;
      if (a.De == 16 && W == 0)
        hipLaunchKernelGGL((k_cluster_expm<T, CPLX, 16>), dim3((unsigned)a.n), dim3(64), 0, s, a);
      else if (a.De == 32 && W == 0)
        hipLaunchKernelGGL((k_cluster_expm<T, CPLX, 32>), dim3((unsigned)a.n), dim3(64), 0, s, a);
      else if (a.De >= 32 && a.De <= 256 && a.expm_scratch != nullptr && a.expm_blocks > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(a.n, a.expm_blocks);
        if (a.De == 32)
          hipLaunchKernelGGL((k_cluster_expm_wg<T, CPLX, 32>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
        else if (a.De == 64)
          hipLaunchKernelGGL((k_cluster_expm_wg<T, CPLX, 64>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
        else if (a.De == 128)
          hipLaunchKernelGGL((k_cluster_expm_wg<T, CPLX, 128>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
        else if (a.De == 256)
          hipLaunchKernelGGL((k_cluster_expm_wg<T, CPLX, 256>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
        else
          return hipErrorInvalidValue;
      } else
        return hipErrorInvalidValue;
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (W == 2) {
    if constexpr (MODE == MODE_CERTIFY && std::is_same<T, double>::value) {
      if ((a.De == 16 || a.De == 32) && a.cert_ws != nullptr) {
        const int G = 64 / a.De;
        if ((a.n + G - 1) / G > 0x7fffffff) return hipErrorInvalidValue;
        const dim3 g1((unsigned)((a.n + G - 1) / G)), g2(grid_for(a.n, 256));
        if (a.De == 16) {
          hipLaunchKernelGGL((k_certify_rows<CPLX, 16>), g1, dim3(64), 0, s, a, a.cert_ws);
          hipLaunchKernelGGL((k_sturm_bisect<16>), g2, dim3(256), 0, s, a, (const double*)a.cert_ws);
        } else {
          hipLaunchKernelGGL((k_certify_rows<CPLX, 32>), g1, dim3(64), 0, s, a, a.cert_ws);
          hipLaunchKernelGGL((k_sturm_bisect<32>), g2, dim3(256), 0, s, a, (const double*)a.cert_ws);
        }
        return hipGetLastError();
      }
      if (a.De == 16 || a.De == 32) {
        if (a.n > 0x7fffffff) return hipErrorInvalidValue;
        if (a.De == 16)
          hipLaunchKernelGGL((k_cluster_tridiag_w<CPLX, 16>), dim3((unsigned)a.n), dim3(64), 0, s, a);
        else
          hipLaunchKernelGGL((k_cluster_tridiag_w<CPLX, 32>), dim3((unsigned)a.n), dim3(64), 0, s, a);
        return hipGetLastError();
      }
      if (a.expm_scratch == nullptr || a.expm_blocks <= 0) return hipErrorInvalidValue;
      const unsigned grid = (unsigned)std::min<int64_t>(a.n, a.expm_blocks);
      // Lanczos + Cholesky certificate at D_e = 256 by default (methods 2 and 3: every D_e >= 64);
      // at 64 and 128 the tridiagonalisation is as fast and its margin tighter
      if (a.cert_method >= 2 || (a.cert_method == 0 && a.De >= 256)) {
        if (a.De == 64)
          hipLaunchKernelGGL((k_certify_lanczos<CPLX, 64>), dim3(grid), dim3(1024), 0, s, a, a.expm_scratch, a.expm_slab);
        else if (a.De == 128)
          hipLaunchKernelGGL((k_certify_lanczos<CPLX, 128>), dim3(grid), dim3(1024), 0, s, a, a.expm_scratch, a.expm_slab);
        else if (a.De == 256)
          hipLaunchKernelGGL((k_certify_lanczos<CPLX, 256>), dim3(grid), dim3(1024), 0, s, a, a.expm_scratch, a.expm_slab);
        else
          return hipErrorInvalidValue;
        return hipGetLastError();
      }
      if (a.De == 64)
        hipLaunchKernelGGL((k_cluster_tridiag<CPLX, 64>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
      else if (a.De == 128)
        hipLaunchKernelGGL((k_cluster_tridiag<CPLX, 128>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
      else if (a.De == 256)
        hipLaunchKernelGGL((k_cluster_tridiag<CPLX, 256>), dim3(grid), dim3(256), 0, s, a, a.expm_scratch, a.expm_slab);
      else
        return hipErrorInvalidValue;
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (W == 5) {   // clusters with a spin-1 site: table-driven Jacobi on the padded dimension
    if (a.gtab == nullptr && a.Dc > 0) return hipErrorInvalidValue;
    const int De = a.De;
    if (De <= 4) hipLaunchKernelGGL((k_cluster_gen<T, CPLX, 4, MODE, 4>), dim3((unsigned)((a.n + 15) / 16)), dim3(64), 0, s, a);
    else if (De <= 8) hipLaunchKernelGGL((k_cluster_gen<T, CPLX, 8, MODE, 8>), dim3((unsigned)((a.n + 7) / 8)), dim3(64), 0, s, a);
    else if (De <= 16) hipLaunchKernelGGL((k_cluster_gen<T, CPLX, 16, MODE, 16>), dim3((unsigned)((a.n + 3) / 4)), dim3(64), 0, s, a);
    else if (De <= 32) hipLaunchKernelGGL((k_cluster_gen<T, CPLX, 32, MODE, 32>), dim3((unsigned)((a.n + 1) / 2)), dim3(64), 0, s, a);
    else if (De <= 64) hipLaunchKernelGGL((k_cluster_gen<T, CPLX, 64, MODE, 64>), dim3((unsigned)a.n), dim3(64), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (W == 1 && a.De >= 8) {
    if (a.De == 8 && a.Dc == 4) return launch_reg<T, CPLX, MODE, 8, 4>(a, block, s);
    if (a.De == 8 && a.Dc == 2) return launch_reg<T, CPLX, MODE, 8, 2>(a, block, s);
    if (a.De == 8 && a.Dc == 0) return launch_reg<T, CPLX, MODE, 8, 0>(a, block, s);
    return hipErrorInvalidValue;
  }
  if (a.De == 2 && a.Dc == 0) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, 2, 0, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
  } else if (a.De == 4 && a.Dc == 2) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, 4, 2, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
  } else if (a.De == 4 && a.Dc == 0 && W == 1) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, 4, 0, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
  } else if (a.fp != nullptr) {
    return hipErrorInvalidValue;  // fused update only in the register kernel
  } else if (a.De == 4 && W == 64) {
    launch_lds_w<T, CPLX, MODE, 4, 64>(a, s);
  } else if (a.De == 8 && W == 16) {
    launch_lds_w<T, CPLX, MODE, 8, 16>(a, s);
  } else if (a.De == 8 && W == 8) {
    launch_lds_w<T, CPLX, MODE, 8, 8>(a, s);
  } else if (a.De == 8 && W == 64) {
    launch_lds_w<T, CPLX, MODE, 8, 64>(a, s);
  } else if (a.De == 16 && W == 16) {
    launch_lds_w<T, CPLX, MODE, 16, 16>(a, s);
  } else if (a.De == 16 && W == 32) {
    launch_lds_w<T, CPLX, MODE, 16, 32>(a, s);
  } else if (a.De == 16 && W == 64) {
    launch_lds_w<T, CPLX, MODE, 16, 64>(a, s);
  } else if (a.De == 32 && W == 32) {
    launch_lds_w<T, CPLX, MODE, 32, 32>(a, s);
  } else if (a.De == 32 && W == 64) {
    launch_lds_w<T, CPLX, MODE, 32, 64>(a, s);
  } else if (a.De == 64 && W == 64) {
    launch_lds_w<T, CPLX, MODE, 64, 64>(a, s);
  } else if ((a.De == 128 || a.De == 256) && a.big_scratch != nullptr) {
    const unsigned grid = (unsigned)std::min<int64_t>(a.n, a.big_blocks);
    hipLaunchKernelGGL((k_cluster_big<T, CPLX, MODE>), dim3(grid), dim3(1024), 0, s, a, (T*)a.big_scratch,
                       a.big_slab);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


// Entry of the cluster kernels for one (precision, field, mode): explicitly instantiated in
// one translation unit each, so that the kernel families compile in parallel.
template <typename T, bool CPLX, int MODE>
hipError_t launch_cluster_mode(const ClusterArgs<T>& a, int block, int W, hipStream_t s) {
  return launch_cluster_m<T, CPLX, MODE>(a, block, W, s);
}

}  // namespace lrh
