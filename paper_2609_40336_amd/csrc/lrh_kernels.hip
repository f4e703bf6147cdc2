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
#include "lrh_internal.h"

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

namespace lrh {

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------

template <typename T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T dexp(T x);
template <> __device__ __forceinline__ float dexp<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double dexp<double>(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T dlog(T x);
template <> __device__ __forceinline__ float dlog<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double dlog<double>(double x) { return log(x); }
template <typename T> __device__ __forceinline__ T dfma(T a, T b, T c);
template <> __device__ __forceinline__ float dfma<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ __forceinline__ double dfma<double>(double a, double b, double c) { return fma(a, b, c); }

// Algorithm 2 extrapolation / averaging (1 - th) x + th y, with one explicit rounding
// pattern so that every kernel computing it from the same inputs gets the same bits.
template <typename T>
__device__ __forceinline__ T extrap(T x, T y, T th) {
  return dfma<T>(T(1) - th, x, th * y);
}

// Jacobi rotation parameters for a pair with (real-ified) off-diagonal magnitude r > 0:
// tau = (a_qq - a_pp) / (2 r), t = sign(tau) / (|tau| + sqrt(tau^2 + 1)), c = 1/sqrt(1+t^2).
template <typename T>
__device__ __forceinline__ void rot_params(T app, T aqq, T r, T& t, T& c, T& s) {
  T tau = (aqq - app) / (T(2) * r);
  T at = fabs(tau);
  t = (tau >= T(0) ? T(1) : T(-1)) / (at + dsqrt<T>(dfma<T>(tau, tau, T(1))));
  c = T(1) / dsqrt<T>(dfma<T>(t, t, T(1)));
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
// register-resident cluster kernel (De <= 4)
// ------------------------------------------------------------------------------------------

template <typename T, bool CPLX, int D, typename Get>
__device__ __forceinline__ void unpack(Get get, T (&xr)[D][D], T (&xi)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T v = get(tri_index(i, j, D));
      xr[i][j] = v;
      xr[j][i] = v;
    }
  if constexpr (CPLX) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xi[i][i] = T(0);
#pragma unroll
      for (int j = i + 1; j < D; ++j) {
        T v = get(D * (D + 1) / 2 + stri_index(i, j, D));
        xi[i][j] = v;
        xi[j][i] = -v;
      }
    }
  }
}

template <typename T, bool CPLX, int D, typename Put>
__device__ __forceinline__ void pack(Put put, const T (&xr)[D][D], const T (&xi)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) put(tri_index(i, j, D), xr[i][j]);
  if constexpr (CPLX) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i + 1; j < D; ++j) put(D * (D + 1) / 2 + stri_index(i, j, D), xi[i][j]);
  }
}

// theta_e -= 1_{e\f} (x) X for a child whose sites occupy bit mask MASK of e's index.
template <typename T, bool CPLX, int DE, int DC, int MASK>
__device__ __forceinline__ void lift_sub(T (&ar)[DE][DE], T (&ai)[DE][DE], const T (&xr)[DC][DC],
                                         const T (&xi)[DC][DC]) {
  constexpr int NB = log2i(DE);
#pragma unroll
  for (int i = 0; i < DE; ++i)
#pragma unroll
    for (int j = 0; j < DE; ++j) {
      if (((i ^ j) & ~MASK & (DE - 1)) == 0) {
        ar[i][j] -= xr[pext_bits(i, MASK, NB)][pext_bits(j, MASK, NB)];
        if constexpr (CPLX) ai[i][j] -= xi[pext_bits(i, MASK, NB)][pext_bits(j, MASK, NB)];
      }
    }
}

// T = Tr_{e\f} rho for a child at mask MASK.
template <typename T, bool CPLX, int DE, int DC, int MASK>
__device__ __forceinline__ void ptrace_reg(const T (&rr)[DE][DE], const T (&ri)[DE][DE],
                                           T (&tr)[DC][DC], T (&ti)[DC][DC]) {
  constexpr int NB = log2i(DE);
  constexpr int NR = DE / DC;
#pragma unroll
  for (int a = 0; a < DC; ++a)
#pragma unroll
    for (int b = 0; b < DC; ++b) {
      T sr = T(0), si = T(0);
#pragma unroll
      for (int x = 0; x < NR; ++x) {
        sr += rr[pdep_bits(a, x, MASK, NB)][pdep_bits(b, x, MASK, NB)];
        if constexpr (CPLX) si += ri[pdep_bits(a, x, MASK, NB)][pdep_bits(b, x, MASK, NB)];
      }
      tr[a][b] = sr;
      ti[a][b] = si;
    }
}

// One cyclic sweep of two-sided Jacobi rotations over all pairs (p < q), row-cyclic order.
template <typename T, bool CPLX, int D, bool VEC>
__device__ __forceinline__ void jacobi_sweep_reg(T (&ar)[D][D], T (&ai)[D][D], T (&ur)[D][D],
                                                 T (&ui)[D][D]) {
#pragma unroll
  for (int p = 0; p < D - 1; ++p)
#pragma unroll
    for (int q = p + 1; q < D; ++q) {
      T xr = ar[p][q];
      T xi = CPLX ? ai[p][q] : T(0);
      T r = CPLX ? dsqrt<T>(dfma<T>(xr, xr, xi * xi)) : fabs(xr);
      if (r != T(0)) {
        T t, c, s;
        // e^{-i phi} with a_pq = r e^{i phi}; real case: sign(a_pq)
        T er = xr / r, ei = CPLX ? -xi / r : T(0);
        rot_params<T>(ar[p][p], ar[q][q], r, t, c, s);
        T app = ar[p][p], aqq = ar[q][q];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          if (k == p || k == q) continue;
          // column update (A G): w = a_kq e^{-i phi}
          T pr = ar[k][p], pi = CPLX ? ai[k][p] : T(0);
          T qr = ar[k][q], qi = CPLX ? ai[k][q] : T(0);
          T wr = CPLX ? (qr * er - qi * ei) : qr * er;
          T wi = CPLX ? (qr * ei + qi * er) : T(0);
          T npr = c * pr - s * wr, npi = c * pi - s * wi;
          T nqr = s * pr + c * wr, nqi = s * pi + c * wi;
          ar[k][p] = npr; ar[p][k] = npr;
          ar[k][q] = nqr; ar[q][k] = nqr;
          if constexpr (CPLX) {
            ai[k][p] = npi; ai[p][k] = -npi;
            ai[k][q] = nqi; ai[q][k] = -nqi;
          }
        }
        ar[p][p] = app - t * r;
        ar[q][q] = aqq + t * r;
        ar[p][q] = T(0); ar[q][p] = T(0);
        if constexpr (CPLX) { ai[p][q] = T(0); ai[q][p] = T(0); }
        if constexpr (VEC) {
#pragma unroll
          for (int k = 0; k < D; ++k) {
            T pr = ur[k][p], pi = CPLX ? ui[k][p] : T(0);
            T qr = ur[k][q], qi = CPLX ? ui[k][q] : T(0);
            T wr = CPLX ? (qr * er - qi * ei) : qr * er;
            T wi = CPLX ? (qr * ei + qi * er) : T(0);
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
}

template <typename T, bool CPLX, int D>
__device__ __forceinline__ T offdiag2(const T (&ar)[D][D], const T (&ai)[D][D]) {
  T s = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (i != j) {
        s = dfma<T>(ar[i][j], ar[i][j], s);
        if constexpr (CPLX) s = dfma<T>(ai[i][j], ai[i][j], s);
      }
  return s;
}

// Loads component k of message m with the Algorithm 2 state handling of this launch:
// plain:  eta = extrap(nu, zeta, theta) (or nu when there is no zeta);
// fused:  first apply the previous iteration's update from (nu, zeta, rho_f, T_{e->f}).
template <typename T>
struct FusedCoef { T thp, ithp, thc; };

template <typename T, bool CPLX, int DE, int DC, int MODE>
__device__ void cluster_reg_body(const ClusterArgs<T>& A, int64_t c) {
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  T ar[DE][DE], ai[DE][DE];
  // ---- a2: h_e ----
  const int64_t ho = A.hoff[c];
  if (ho >= 0) {
    const double* h = A.h + ho;
    unpack<T, CPLX, DE>([&](int k) { return (T)h[k]; }, ar, ai);
  } else {
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = 0; j < DE; ++j) { ar[i][j] = T(0); ai[i][j] = T(0); }
  }
  const bool fused = (A.fp != nullptr);
  FusedCoef<T> fc{};
  if (fused) {
    fc.thp = (T)A.fp->theta_prev;
    fc.ithp = (T)A.fp->inv_thL_prev;
    fc.thc = (T)A.fp->theta_cur;
  }
  const T th = fused ? fc.thc : (T)A.theta;
  // ---- children: subtract lifted messages ----
  if constexpr (DC > 0) {
    for (int s = 0; s < A.maxch; ++s) {
      const int m = A.ch[(int64_t)s * A.n + c];
      if (m < 0) continue;
      const int mask = A.chmask[(int64_t)s * A.n + c];
      T xr[DC][DC], xi[DC][DC];
      if (fused) {
        const int64_t rs = A.rslot_of_msg_c[m];
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
        }, xr, xi);
      } else if (A.ze_c) {
        unpack<T, CPLX, DC>([&](int k) {
          const int64_t o = (int64_t)k * A.Mc + m;
          return extrap<T>(A.nu_c[o], A.ze_c[o], th);
        }, xr, xi);
      } else {
        unpack<T, CPLX, DC>([&](int k) { return A.nu_c[(int64_t)k * A.Mc + m]; }, xr, xi);
      }
      if constexpr (DE == 4 && DC == 2) {
        if (mask == 2) lift_sub<T, CPLX, DE, DC, 2>(ar, ai, xr, xi);
        else lift_sub<T, CPLX, DE, DC, 1>(ar, ai, xr, xi);
      }
    }
  }
  // ---- parents: add messages received ----
  const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
  for (int s = 0; s < A.maxpar; ++s) {
    const int m = A.par[(int64_t)s * A.n + c];
    if (m < 0) continue;
    T xr[DE][DE], xi[DE][DE];
    if (fused) {
      unpack<T, CPLX, DE>([&](int k) {
        const int64_t o = (int64_t)k * A.Mp + m;
        T nu0 = A.nu_p_prev[o], ze0 = A.ze_p_prev[o];
        if (!A.fused_first) {
          T g = A.Rprev_p[(int64_t)k * A.S + rs_self] - A.Tprev_p[o];
          ze0 = dfma<T>(g, fc.ithp, ze0);
          nu0 = extrap<T>(nu0, ze0, fc.thp);
        }
        return extrap<T>(nu0, ze0, th);
      }, xr, xi);
    } else if (A.ze_p) {
      unpack<T, CPLX, DE>([&](int k) {
        const int64_t o = (int64_t)k * A.Mp + m;
        return extrap<T>(A.nu_p[o], A.ze_p[o], th);
      }, xr, xi);
    } else {
      unpack<T, CPLX, DE>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, xr, xi);
    }
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = 0; j < DE; ++j) {
        ar[i][j] += xr[i][j];
        if constexpr (CPLX) ai[i][j] += xi[i][j];
      }
  }
  // ---- a3: cyclic Jacobi ----
  T nrm2 = T(0);
#pragma unroll
  for (int i = 0; i < DE; ++i)
#pragma unroll
    for (int j = 0; j < DE; ++j) {
      nrm2 = dfma<T>(ar[i][j], ar[i][j], nrm2);
      if constexpr (CPLX) nrm2 = dfma<T>(ai[i][j], ai[i][j], nrm2);
    }
  T ur[DE][DE], ui[DE][DE];
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = 0; j < DE; ++j) { ur[i][j] = (i == j) ? T(1) : T(0); ui[i][j] = T(0); }
  }
  const T tol2 = (T)(A.tol * A.tol) * nrm2;
  bool conv = false;
  for (int sweep = 0; sweep <= A.max_sweeps; ++sweep) {
    if (offdiag2<T, CPLX, DE>(ar, ai) <= tol2) { conv = true; break; }
    if (sweep == A.max_sweeps) break;
    jacobi_sweep_reg<T, CPLX, DE, VEC>(ar, ai, ur, ui);
  }
  if (!conv && A.noconv) atomicAdd(A.noconv, 1ull);
  T lam[DE];
  T lmin = ar[0][0];
#pragma unroll
  for (int k = 0; k < DE; ++k) { lam[k] = ar[k][k]; lmin = fmin(lmin, lam[k]); }
  if (!isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  const int32_t gid = A.gid[c];
  if constexpr (MODE == MODE_CERTIFY) {
    A.scal[gid] = (double)lmin;
    A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt((double)nrm2);
    return;
  } else {
    // ---- a4: marginal weights ----
    T p[DE];
    if constexpr (MODE == MODE_GIBBS) {
      // fused launches are replayed from a graph across stages: beta comes from the table
      const T b = fused ? (T)A.fp->beta : (T)A.beta;
      T Z = T(0);
#pragma unroll
      for (int k = 0; k < DE; ++k) { p[k] = dexp<T>(-b * (lam[k] - lmin)); Z += p[k]; }
      const T iZ = T(1) / Z;
#pragma unroll
      for (int k = 0; k < DE; ++k) p[k] *= iZ;
      A.scal[gid] = (double)(lmin - dlog<T>(Z) / b);
    } else {
      const T tau = (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2));
      T g = T(0);
#pragma unroll
      for (int k = 0; k < DE; ++k) { p[k] = (lam[k] <= lmin + tau) ? T(1) : T(0); g += p[k]; }
      const T ig = T(1) / g;
#pragma unroll
      for (int k = 0; k < DE; ++k) p[k] *= ig;
      A.scal[gid] = (double)lmin;
    }
    // rho = U diag(p) U^H  (reuse ar/ai)
#pragma unroll
    for (int i = 0; i < DE; ++i)
#pragma unroll
      for (int j = i; j < DE; ++j) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < DE; ++k) {
          T a_r = ur[i][k] * p[k], a_i = CPLX ? ui[i][k] * p[k] : T(0);
          // (a_r + i a_i) * conj(u_jk)
          sr = dfma<T>(a_r, ur[j][k], sr);
          if constexpr (CPLX) {
            sr = dfma<T>(a_i, ui[j][k], sr);
            si = dfma<T>(a_i, ur[j][k], si);
            si = dfma<T>(-a_r, ui[j][k], si);
          }
        }
        ar[i][j] = sr; ar[j][i] = sr;
        if constexpr (CPLX) { ai[i][j] = si; ai[j][i] = (i == j) ? T(0) : -si; }
      }
    if constexpr (CPLX) {
#pragma unroll
      for (int i = 0; i < DE; ++i) ai[i][i] = T(0);
    }
    // ---- outputs: own marginal ----
    if (rs_self >= 0 && A.R) {
      pack<T, CPLX, DE>([&](int k, T v) { A.R[(int64_t)k * A.S + rs_self] = v; }, ar, ai);
    }
    if (A.marg) {
      T* mo = A.marg + A.marg_off[gid];
      pack<T, CPLX, DE>([&](int k, T v) { mo[k] = v; }, ar, ai);
    }
    // ---- a5: partial traces onto the children ----
    if constexpr (DC > 0) {
      if (A.Tout) {
        for (int s = 0; s < A.maxch; ++s) {
          const int m = A.ch[(int64_t)s * A.n + c];
          if (m < 0) continue;
          const int mask = A.chmask[(int64_t)s * A.n + c];
          T tr[DC][DC], ti[DC][DC];
          if constexpr (DE == 4 && DC == 2) {
            if (mask == 2) ptrace_reg<T, CPLX, DE, DC, 2>(ar, ai, tr, ti);
            else ptrace_reg<T, CPLX, DE, DC, 1>(ar, ai, tr, ti);
          }
          pack<T, CPLX, DC>([&](int k, T v) { A.Tout[(int64_t)k * A.Mc + m] = v; }, tr, ti);
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

template <typename T, bool CPLX, int DE, int MODE>
__global__ __launch_bounds__(64) void k_cluster_lds(ClusterArgs<T> A) {
  constexpr int LD = DE + 1;
  constexpr bool VEC = (MODE != MODE_CERTIFY);
  constexpr int NP = DE / 2;
  constexpr int NB = log2i(DE);
  __shared__ T sar[DE * LD];
  __shared__ T sai[CPLX ? DE * LD : 1];
  __shared__ T sur[VEC ? DE * LD : 1];
  __shared__ T sui[(VEC && CPLX) ? DE * LD : 1];
  __shared__ T cs_c[NP], cs_s[NP], cs_er[NP], cs_ei[NP], cs_app[NP], cs_aqq[NP];
  __shared__ int cs_p[NP], cs_q[NP];
  __shared__ T sp[DE];
  const int64_t c = blockIdx.x;
  if (c >= A.n) return;
  const int tid = threadIdx.x;
  const T th = (T)A.theta;
  const int64_t ho = A.hoff[c];
  const int Dc = A.Dc;
  // ---- a2: assemble theta_e ----
  T my_n2 = T(0);
  for (int idx = tid; idx < DE * DE; idx += 64) {
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
                                  return extrap<T>(A.nu_p[o], A.ze_p[o], th); }, i, j, DE, CPLX, er, ei);
      else
        herm_elem<T>([&](int k) { return A.nu_p[(int64_t)k * A.Mp + m]; }, i, j, DE, CPLX, er, ei);
      vr += er;
      vi += ei;
    }
    sar[i * LD + j] = vr;
    if constexpr (CPLX) sai[i * LD + j] = vi;
    if constexpr (VEC) {
      sur[i * LD + j] = (i == j) ? T(1) : T(0);
      if constexpr (CPLX) sui[i * LD + j] = T(0);
    }
    my_n2 = dfma<T>(vr, vr, my_n2);
    if constexpr (CPLX) my_n2 = dfma<T>(vi, vi, my_n2);
  }
  const T nrm2 = wave_sum(my_n2);
  __syncthreads();
  // ---- a3: parallel cyclic Jacobi (round-robin ordering) ----
  const T tol2 = (T)(A.tol * A.tol) * nrm2;
  bool conv = false;
  for (int sweep = 0; sweep <= A.max_sweeps; ++sweep) {
    T off = T(0);
    for (int idx = tid; idx < DE * DE; idx += 64) {
      const int i = idx / DE, j = idx % DE;
      if (i != j) {
        off = dfma<T>(sar[i * LD + j], sar[i * LD + j], off);
        if constexpr (CPLX) off = dfma<T>(sai[i * LD + j], sai[i * LD + j], off);
      }
    }
    off = wave_sum(off);
    if (off <= tol2) { conv = true; break; }
    if (sweep == A.max_sweeps) break;
    for (int r = 0; r < DE - 1; ++r) {
      if (tid < NP) {
        int p, q;
        rr_pair(r, tid, DE, p, q);
        const T xr = sar[p * LD + q];
        const T xi = CPLX ? sai[p * LD + q] : T(0);
        const T rr = CPLX ? dsqrt<T>(dfma<T>(xr, xr, xi * xi)) : fabs(xr);
        T t = T(0), cc = T(1), ss = T(0), er = T(1), ei = T(0);
        const T app = sar[p * LD + p], aqq = sar[q * LD + q];
        if (rr != T(0)) {
          rot_params<T>(app, aqq, rr, t, cc, ss);
          er = xr / rr;
          ei = CPLX ? -xi / rr : T(0);
        }
        cs_p[tid] = p; cs_q[tid] = q;
        cs_c[tid] = cc; cs_s[tid] = ss; cs_er[tid] = er; cs_ei[tid] = ei;
        cs_app[tid] = app - t * rr;
        cs_aqq[tid] = aqq + t * rr;
      }
      __syncthreads();
      // columns: A <- A G, U <- U G  (w = x_q e^{-i phi})
      for (int idx = tid; idx < DE * NP; idx += 64) {
        const int i = idx % DE, k = idx / DE;
        const int p = cs_p[k], q = cs_q[k];
        const T cc = cs_c[k], ss = cs_s[k], er = cs_er[k], ei = cs_ei[k];
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
      __syncthreads();
      // rows: A <- G^H A  (w = x_q e^{+i phi})
      for (int idx = tid; idx < DE * NP; idx += 64) {
        const int j = idx % DE, k = idx / DE;
        const int p = cs_p[k], q = cs_q[k];
        const T cc = cs_c[k], ss = cs_s[k], er = cs_er[k], ei = -cs_ei[k];
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
      __syncthreads();
      if (tid < NP) {
        const int p = cs_p[tid], q = cs_q[tid];
        sar[p * LD + p] = cs_app[tid];
        sar[q * LD + q] = cs_aqq[tid];
        sar[p * LD + q] = T(0);
        sar[q * LD + p] = T(0);
        if constexpr (CPLX) {
          sai[p * LD + p] = T(0); sai[q * LD + q] = T(0);
          sai[p * LD + q] = T(0); sai[q * LD + p] = T(0);
        }
      }
      __syncthreads();
    }
  }
  if (!conv && tid == 0 && A.noconv) atomicAdd(A.noconv, 1ull);
  // ---- eigenvalues ----
  T lmin = T(INFINITY);
  for (int k = tid; k < DE; k += 64) lmin = fmin(lmin, sar[k * LD + k]);
  lmin = wave_min(lmin);
  if (tid == 0 && !isfinite((double)lmin) && A.nonfinite) atomicAdd(A.nonfinite, 1ull);
  const int32_t gid = A.gid[c];
  if constexpr (MODE == MODE_CERTIFY) {
    if (tid == 0) {
      A.scal[gid] = (double)lmin;
      A.scal2[gid] = 8.0 * DE * DBL_EPSILON * sqrt((double)nrm2);
    }
    return;
  } else {
    // ---- a4: weights ----
    T w = T(0);
    if constexpr (MODE == MODE_GIBBS) {
      const T b = (T)A.beta;
      for (int k = tid; k < DE; k += 64) { T v = dexp<T>(-b * (sar[k * LD + k] - lmin)); sp[k] = v; w += v; }
      const T Z = wave_sum(w);
      __syncthreads();
      for (int k = tid; k < DE; k += 64) sp[k] /= Z;
      if (tid == 0) A.scal[gid] = (double)(lmin - dlog<T>(Z) / b);
    } else {
      const T tau = (T)A.tau_rel * fmax(T(1), dsqrt<T>(nrm2));
      for (int k = tid; k < DE; k += 64) { T v = (sar[k * LD + k] <= lmin + tau) ? T(1) : T(0); sp[k] = v; w += v; }
      const T g = wave_sum(w);
      __syncthreads();
      for (int k = tid; k < DE; k += 64) sp[k] /= g;
      if (tid == 0) A.scal[gid] = (double)lmin;
    }
    __syncthreads();
    // rho = U diag(p) U^H, written over A
    for (int idx = tid; idx < DE * DE; idx += 64) {
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
      sar[i * LD + j] = sr;
      if constexpr (CPLX) sai[i * LD + j] = (i == j) ? T(0) : si;
    }
    __syncthreads();
    // ---- outputs ----
    const int64_t rs_self = A.rslot ? A.rslot[c] : -1;
    constexpr int NCE = n_comps(DE, CPLX);
    for (int k = tid; k < NCE; k += 64) {
      // decode component k -> (i, j)
      int i = 0, j = 0;
      bool im = false;
      int kk = k;
      if (kk >= DE * (DE + 1) / 2) { im = true; kk -= DE * (DE + 1) / 2; }
      const int rowlen0 = im ? DE - 1 : DE;
      while (kk >= rowlen0 - i) { kk -= rowlen0 - i; ++i; }
      j = i + kk + (im ? 1 : 0);
      const T v = im ? sai[i * LD + j] : sar[i * LD + j];
      if (rs_self >= 0 && A.R) A.R[(int64_t)k * A.S + rs_self] = v;
      if (A.marg) A.marg[A.marg_off[gid] + k] = v;
    }
    if (A.Tout && Dc > 0) {
      const int NR = DE / Dc;
      const int NCC = CPLX ? Dc * Dc : Dc * (Dc + 1) / 2;
      for (int s = 0; s < A.maxch; ++s) {
        const int m = A.ch[(int64_t)s * A.n + c];
        if (m < 0) continue;
        const int mask = A.chmask[(int64_t)s * A.n + c];
        for (int k = tid; k < NCC; k += 64) {
          int a = 0, b = 0;
          bool im = false;
          int kk = k;
          if (kk >= Dc * (Dc + 1) / 2) { im = true; kk -= Dc * (Dc + 1) / 2; }
          const int rowlen0 = im ? Dc - 1 : Dc;
          while (kk >= rowlen0 - a) { kk -= rowlen0 - a; ++a; }
          b = a + kk + (im ? 1 : 0);
          T sum = T(0);
          for (int x = 0; x < NR; ++x) {
            const int i = pdep_rt(a, x, mask, NB), j = pdep_rt(b, x, mask, NB);
            sum += im ? sai[i * LD + j] : sar[i * LD + j];
          }
          A.Tout[(int64_t)k * A.Mc + m] = sum;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// message kernel (a6), reductions, small helpers
// ------------------------------------------------------------------------------------------

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_msg(MsgArgs<T> A) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= A.M) return;
  const int64_t rs = A.rslot[m];
  T th, ith;
  if (A.fp) { th = (T)A.fp->theta_prev; ith = (T)A.fp->inv_thL_prev; }
  else { th = (T)A.theta; ith = (T)A.inv_thL; }
  const bool copy_best = (MODE == MSG_SUBGRAD) && A.improved && A.improved[A.inst[m]];
  const T alpha = (T)A.alpha;
  const T* nsrc = A.nu_src ? A.nu_src : A.nu;
  const T* zsrc = A.ze_src ? A.ze_src : A.ze;
  for (int64_t k = 0; k < A.comps; ++k) {
    const int64_t o = k * A.M + m;
    const T g = A.R[k * A.S + rs] - A.Tm[o];
    if constexpr (MODE == MSG_GRAD) {
      A.grad[o] = g;
    } else if constexpr (MODE == MSG_SUBGRAD) {
      const T v = nsrc[o];
      if (copy_best) A.nu_best[o] = v;
      A.nu[o] = dfma<T>(alpha, g, v);
    } else {
      const T z = dfma<T>(g, ith, zsrc[o]);
      A.ze[o] = z;
      A.nu[o] = extrap<T>(nsrc[o], z, th);
    }
  }
}

// Per-instance sums over the contiguous library-cluster range of each instance, in a fixed
// order (strided per-thread partial sums, then a fixed tree): bitwise reproducible.
__global__ __launch_bounds__(256) void k_reduce(const double* scal, const int64_t* ptr, double* out,
                                                const double* scal2, double* out2, double* q_best,
                                                int32_t* improved, double* q_hist) {
  __shared__ double sh[256];
  __shared__ double sh2[256];
  const int i = blockIdx.x;
  const int64_t a = ptr[i], b = ptr[i + 1];
  double s = 0.0, s2 = 0.0;
  for (int64_t j = a + threadIdx.x; j < b; j += 256) {
    s += scal[j];
    if (scal2) s2 += scal2[j];
  }
  sh[threadIdx.x] = s;
  sh2[threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[threadIdx.x] += sh[threadIdx.x + w];
      sh2[threadIdx.x] += sh2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double q = sh[0];
    if (out) out[i] = q;
    if (out2) out2[i] = sh2[0];
    if (q_hist) q_hist[i] = q;
    if (q_best) {
      const bool better = q > q_best[i];
      improved[i] = better ? 1 : 0;
      if (better) q_best[i] = q;
    }
  }
}

__global__ void k_set_fused(FusedParams* dst, FusedTable v, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = v.p[i];
}

__global__ __launch_bounds__(256) void k_widen(double* dst, const float* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// Edges and sites of a 2-local problem in one launch: blocks [0, nbe) take edges, the rest
// take sites.  Both buckets read only the previous iteration's buffers, so they need no
// ordering between them.
template <typename T, bool CPLX, int MODE>
__global__ __launch_bounds__(256) void k_cluster_pair(ClusterArgs<T> E, ClusterArgs<T> S, int nbe) {
  if ((int)blockIdx.x < nbe) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < E.n) cluster_reg_body<T, CPLX, 4, 2, MODE>(E, c);
  } else {
    const int64_t c = (int64_t)(blockIdx.x - nbe) * blockDim.x + threadIdx.x;
    if (c < S.n) cluster_reg_body<T, CPLX, 2, 0, MODE>(S, c);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(T* dst, const T* src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <typename T, bool CPLX, int MODE>
static hipError_t launch_cluster_m(const ClusterArgs<T>& a, int block, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (a.De == 2 && a.Dc == 0) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, 2, 0, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
  } else if (a.De == 4 && a.Dc == 2) {
    hipLaunchKernelGGL((k_cluster_reg<T, CPLX, 4, 2, MODE>), dim3(grid_for(a.n, block)), dim3(block), 0, s, a);
  } else if (a.fp != nullptr) {
    return hipErrorInvalidValue;  // fused update only in the register kernel
  } else if (a.De == 4) {
    hipLaunchKernelGGL((k_cluster_lds<T, CPLX, 4, MODE>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  } else if (a.De == 8) {
    hipLaunchKernelGGL((k_cluster_lds<T, CPLX, 8, MODE>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  } else if (a.De == 16) {
    hipLaunchKernelGGL((k_cluster_lds<T, CPLX, 16, MODE>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  } else if (a.De == 32) {
    hipLaunchKernelGGL((k_cluster_lds<T, CPLX, 32, MODE>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  } else if (a.De == 64) {
    hipLaunchKernelGGL((k_cluster_lds<T, CPLX, 64, MODE>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cluster(const ClusterArgs<T>& a, bool cplx, int mode, int block, hipStream_t s) {
  if (mode == MODE_CERTIFY) {
    if constexpr (std::is_same<T, double>::value) {
      return cplx ? launch_cluster_m<T, true, MODE_CERTIFY>(a, block, s)
                  : launch_cluster_m<T, false, MODE_CERTIFY>(a, block, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (mode == MODE_GIBBS)
    return cplx ? launch_cluster_m<T, true, MODE_GIBBS>(a, block, s)
                : launch_cluster_m<T, false, MODE_GIBBS>(a, block, s);
  return cplx ? launch_cluster_m<T, true, MODE_GROUND>(a, block, s)
              : launch_cluster_m<T, false, MODE_GROUND>(a, block, s);
}

template <typename T>
hipError_t launch_msg(const MsgArgs<T>& a, int mode, int block, hipStream_t s) {
  if (a.M == 0) return hipSuccess;
  const dim3 g(grid_for(a.M, block)), b(block);
  if (mode == MSG_GRAD) hipLaunchKernelGGL((k_msg<T, MSG_GRAD>), g, b, 0, s, a);
  else if (mode == MSG_SUBGRAD) hipLaunchKernelGGL((k_msg<T, MSG_SUBGRAD>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_msg<T, MSG_NESTEROV>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* scal, const int64_t* inst_ptr, int64_t n_inst, double* out,
                         const double* scal2, double* out2, double* q_best, int32_t* improved,
                         double* q_hist, hipStream_t s) {
  if (n_inst == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)n_inst), dim3(256), 0, s, scal, inst_ptr, out, scal2,
                     out2, q_best, improved, q_hist);
  return hipGetLastError();
}

hipError_t launch_set_fused(FusedParams* dst, const FusedTable& v, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_fused, dim3(1), dim3(64), 0, s, dst, v, n);
  return hipGetLastError();
}

hipError_t launch_widen(double* dst, const float* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cluster_pair(const ClusterArgs<T>& e, const ClusterArgs<T>& st, bool cplx, int mode,
                               int block, hipStream_t s) {
  const int nbe = (int)grid_for(e.n, block), nbs = (int)grid_for(st.n, block);
  if (nbe + nbs == 0) return hipSuccess;
  const dim3 g(nbe + nbs), b(block);
  if (mode == MODE_GIBBS) {
    if (cplx) hipLaunchKernelGGL((k_cluster_pair<T, true, MODE_GIBBS>), g, b, 0, s, e, st, nbe);
    else hipLaunchKernelGGL((k_cluster_pair<T, false, MODE_GIBBS>), g, b, 0, s, e, st, nbe);
  } else if (mode == MODE_GROUND) {
    if (cplx) hipLaunchKernelGGL((k_cluster_pair<T, true, MODE_GROUND>), g, b, 0, s, e, st, nbe);
    else hipLaunchKernelGGL((k_cluster_pair<T, false, MODE_GROUND>), g, b, 0, s, e, st, nbe);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template hipError_t launch_cluster<float>(const ClusterArgs<float>&, bool, int, int, hipStream_t);
template hipError_t launch_cluster<double>(const ClusterArgs<double>&, bool, int, int, hipStream_t);
template hipError_t launch_msg<float>(const MsgArgs<float>&, int, int, hipStream_t);
template hipError_t launch_msg<double>(const MsgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_copy<float>(float*, const float*, int64_t, hipStream_t);
template hipError_t launch_cluster_pair<float>(const ClusterArgs<float>&, const ClusterArgs<float>&, bool, int, int,
                                               hipStream_t);
template hipError_t launch_cluster_pair<double>(const ClusterArgs<double>&, const ClusterArgs<double>&, bool, int,
                                                int, hipStream_t);
template hipError_t launch_copy<double>(double*, const double*, int64_t, hipStream_t);

}  // namespace lrh
