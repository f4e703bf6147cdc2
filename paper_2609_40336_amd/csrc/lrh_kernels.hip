// Launchers of the cluster kernels (dispatch by precision, field and mode), the message,
// reduction and element-wise kernels.  The cluster kernel families themselves are instantiated
// in lrh_k_*.hip (one translation unit per precision and mode).
#include "lrh_device.h"

namespace lrh {

// ------------------------------------------------------------------------------------------
// message kernel (a6), reductions, small helpers
// ------------------------------------------------------------------------------------------

// message components per thread of the update kernel: the whole message for one- and two-site
// messages with 3, 4 or 10 components, else chunks of 16
constexpr int kMsgChunk = 16;

template <typename T, int MODE, int CH>
__global__ __launch_bounds__(256) void k_msg(MsgArgs<T> A) {
  // x: one thread per message; y: chunks of CH components, so that buckets of large messages
  // (few messages, up to 65536 components each) still fill the GPU
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= A.M) return;
  const int64_t k0 = (int64_t)blockIdx.y * CH;
  const int64_t k1 = k0 + CH < A.comps ? k0 + CH : A.comps;
  const int64_t rs = A.rslot[m];
  T th, ith;
  if (A.fp && A.fp_cur) { th = (T)A.fp->theta_cur; ith = (T)A.fp->inv_thL_cur; }
  else if (A.fp) { th = (T)A.fp->theta_prev; ith = (T)A.fp->inv_thL_prev; }
  else { th = (T)A.theta; ith = (T)A.inv_thL; }
  const bool copy_best = (MODE == MSG_SUBGRAD) && A.improved && A.improved[A.inst[m]];
  const T alpha = (T)A.alpha;
  const T* nsrc = A.nu_src ? A.nu_src : A.nu;
  const T* zsrc = A.ze_src ? A.ze_src : A.ze;
  // Every load of the chunk is issued before the first store, so that a thread keeps up to
  // 4 x CH reads in flight; the message's own entries come first, since they do not wait for
  // the marginal slot.  Loads past the chunk's end (k1 - k0 is the same across a workgroup)
  // repeat its last component, so that none of them sits behind a branch.
  const int64_t nk = k1 - k0;  // 1 .. CH
  T rv[CH], tv[CH], nv[CH], zv[CH];
#pragma unroll
  for (int kk = 0; kk < CH; ++kk) {
    const int64_t k = k0 + (kk < nk ? kk : nk - 1);
    const int64_t o = k * A.M + m;
    tv[kk] = A.Tm[o];
    if constexpr (MODE != MSG_GRAD) nv[kk] = nsrc[o];
    if constexpr (MODE == MSG_NESTEROV) zv[kk] = zsrc[o];
  }
#pragma unroll
  for (int kk = 0; kk < CH; ++kk) {
    const int64_t k = k0 + (kk < nk ? kk : nk - 1);
    rv[kk] = A.R[k * A.S + rs];
  }
#pragma unroll
  for (int kk = 0; kk < CH; ++kk) {
    const int64_t k = k0 + kk;
    if (kk < nk) {
      const int64_t o = k * A.M + m;
      const T g = rv[kk] - tv[kk];
      if constexpr (MODE == MSG_GRAD) {
        A.grad[o] = g;
      } else if constexpr (MODE == MSG_SUBGRAD) {
        const T v = nv[kk];
        if (copy_best) A.nu_best[o] = v;
        A.nu[o] = dfma<T>(alpha, g, v);
      } else {
        const T z = dfma<T>(g, ith, zv[kk]);
        A.ze[o] = z;
        A.nu[o] = extrap<T>(nv[kk], z, th);
      }
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

template <typename T>
__global__ __launch_bounds__(256) void k_fill_noise(T* x, int64_t n, double scale, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // splitmix64 finaliser of (seed, i)
  uint64_t z = ((uint64_t)seed << 32) ^ (uint64_t)i;
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
  x[i] = (T)(scale * (2.0 * u - 1.0));
}

template <typename T>
__global__ __launch_bounds__(256) void k_extrap(T* dst, const T* nu, const T* ze, double th, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = extrap<T>(nu[i], ze[i], (T)th);
}

__global__ __launch_bounds__(256) void k_set_params(double* h, const double* hfix, const int64_t* pc_hoff,
                                                    const int64_t* pc_ptr, const int32_t* pc_param,
                                                    const int64_t* pc_doff, const double* dterm,
                                                    const int32_t* pc_ncomp, int64_t n_pc, const double* params) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_pc) return;
  const int64_t ho = pc_hoff[c];
  const int nc = pc_ncomp[c];
  for (int k = 0; k < nc; ++k) {
    double v = hfix[ho + k];
    for (int64_t t = pc_ptr[c]; t < pc_ptr[c + 1]; ++t) v = fma(params[pc_param[t]], dterm[pc_doff[t] + k], v);
    h[ho + k] = v;
  }
}

// <Y, B> for packed Hermitian D x D matrices: diagonal once, off-diagonal (real and imaginary) twice.
__device__ __forceinline__ double packed_inner(const double* y, const double* b, int D, bool cplx) {
  double s = 0.0;
  int k = 0;
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j, ++k) s = fma((i == j) ? 1.0 : 2.0, y[k] * b[k], s);
  if (cplx) {
    const int n = D * (D - 1) / 2;
    for (int q = 0; q < n; ++q, ++k) s = fma(2.0, y[k] * b[k], s);
  }
  return s;
}

__global__ __launch_bounds__(256) void k_param_bar(double* out, int accumulate, int64_t n_params,
                                                   const int64_t* pp_ptr, const int64_t* pp_yoff,
                                                   const int64_t* pp_doff, const int32_t* pp_D, const double* Y,
                                                   const double* dterm, int cplx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_params) return;
  double s = 0.0;
  for (int64_t t = pp_ptr[p]; t < pp_ptr[p + 1]; ++t)
    s += packed_inner(Y + pp_yoff[t], dterm + pp_doff[t], pp_D[t], cplx != 0);
  out[p] = accumulate ? out[p] + s : s;
}

__global__ __launch_bounds__(256) void k_adj_pre(const double* a, const double* b, double* btot, double* gbar,
                                                 double th, double invthL, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double bt = fma(th, a[i], b[i]);
  btot[i] = bt;
  gbar[i] = bt * invthL;
}

__global__ __launch_bounds__(256) void k_adj_post(double* a, double* b, const double* btot, const double* etabar,
                                                  double th, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  a[i] = (1.0 - th) * (a[i] + etabar[i]);
  b[i] = fma(th, etabar[i], btot[i]);
}

__global__ __launch_bounds__(256) void k_scale_offdiag(double* x, int64_t M, int D, int cplx, double f) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int k = 0;
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j, ++k)
      if (i != j) x[(int64_t)k * M + m] *= f;
  if (cplx) {
    const int n = D * (D - 1) / 2;
    for (int q = 0; q < n; ++q, ++k) x[(int64_t)k * M + m] *= f;
  }
}


// Sustained FP64 matrix-core rate: every lane runs 8 independent chains of
// v_mfma_f64_16x16x4_f64 (2048 flops each per wave); out receives one value per thread.
__global__ __launch_bounds__(256) void k_mfma_f64_rate(double* out, int iters, double seed) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 c[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) c[i] = d4{0.0, 0.0, 0.0, 0.0};
  const double a = seed + threadIdx.x, b = 0.5 * seed;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) r += c[i][0] + c[i][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

hipError_t launch_mfma_f64_rate(double* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_f64_rate, dim3((unsigned)blocks), dim3(256), 0, s, out, iters, 1e-3);
  return hipGetLastError();
}

int cluster_shapes(int De, int Dc, bool dbl, bool cplx, int mode, int* out) {
  int n = 0;
  if ((De & (De - 1)) != 0) {   // a spin-1 site: the table-driven kernel only
    if (De <= 64) out[n++] = 5;
    return n;
  }
  bool reg = reg_pair(De, Dc);
  if (reg && De >= 8) {
    if (De == 8) reg = !(dbl && cplx && mode != MODE_CERTIFY);
  }
  if (reg) out[n++] = 1;
  if (mode == MODE_GIBBS && expm_ok(De, cplx)) {
    if (De <= 32) out[n++] = 0;   // one wave per cluster
    if (De >= 32) out[n++] = 4;   // one workgroup per cluster
  }
  if (mode == MODE_CERTIFY && De >= 16 && De <= 256) out[n++] = 2;
  int lds[8];
  const int nl = lds_shapes(De, lds);
  if (!(De <= 4 && reg))
    for (int i = 0; i < nl; ++i) out[n++] = lds[i];
  return n;
}

// LDS shapes compiled per dimension (lanes per cluster); the first is the default.
int lds_shapes(int De, int* out) {
  switch (De) {
    case 4: out[0] = 64; return 1;
    case 8: out[0] = 16; out[1] = 8; out[2] = 64; return 3;
    case 16: out[0] = 16; out[1] = 32; out[2] = 64; return 3;
    case 32: out[0] = 32; out[1] = 64; return 2;
    case 64: out[0] = 64; return 1;
    case 128: out[0] = 1024; return 1;
    case 256: out[0] = 1024; return 1;
    default: return 0;
  }
}

extern template hipError_t launch_cluster_mode<float, false, MODE_GIBBS>(const ClusterArgs<float>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<float, true, MODE_GIBBS>(const ClusterArgs<float>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<float, false, MODE_GROUND>(const ClusterArgs<float>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<float, true, MODE_GROUND>(const ClusterArgs<float>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, false, MODE_GIBBS>(const ClusterArgs<double>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, true, MODE_GIBBS>(const ClusterArgs<double>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, false, MODE_GROUND>(const ClusterArgs<double>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, true, MODE_GROUND>(const ClusterArgs<double>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, false, MODE_CERTIFY>(const ClusterArgs<double>&, int, int, hipStream_t);
extern template hipError_t launch_cluster_mode<double, true, MODE_CERTIFY>(const ClusterArgs<double>&, int, int, hipStream_t);

template <typename T>
hipError_t launch_cluster(const ClusterArgs<T>& a, bool cplx, int mode, int block, int W, hipStream_t s) {
  if (mode == MODE_CERTIFY) {
    if constexpr (std::is_same<T, double>::value) {
      return cplx ? launch_cluster_mode<T, true, MODE_CERTIFY>(a, block, W, s)
                  : launch_cluster_mode<T, false, MODE_CERTIFY>(a, block, W, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (mode == MODE_GIBBS)
    return cplx ? launch_cluster_mode<T, true, MODE_GIBBS>(a, block, W, s)
                : launch_cluster_mode<T, false, MODE_GIBBS>(a, block, W, s);
  return cplx ? launch_cluster_mode<T, true, MODE_GROUND>(a, block, W, s)
              : launch_cluster_mode<T, false, MODE_GROUND>(a, block, W, s);
}

template <typename T>
hipError_t launch_msg(const MsgArgs<T>& a, int mode, int block, hipStream_t s) {
  if (a.M == 0 || a.comps == 0) return hipSuccess;
  const int ch = (a.comps == 3 || a.comps == 4 || a.comps == 10) ? (int)a.comps : kMsgChunk;
  const int64_t chunks = (a.comps + ch - 1) / ch;
  if (chunks > 65535) return hipErrorInvalidValue;
  const dim3 g(grid_for(a.M, block), (unsigned)chunks), b(block);
  auto go = [&](auto chc) {
    constexpr int CH = decltype(chc)::value;
    if (mode == MSG_GRAD) hipLaunchKernelGGL((k_msg<T, MSG_GRAD, CH>), g, b, 0, s, a);
    else if (mode == MSG_SUBGRAD) hipLaunchKernelGGL((k_msg<T, MSG_SUBGRAD, CH>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_msg<T, MSG_NESTEROV, CH>), g, b, 0, s, a);
  };
  if (ch == 3) go(std::integral_constant<int, 3>{});
  else if (ch == 4) go(std::integral_constant<int, 4>{});
  else if (ch == 10) go(std::integral_constant<int, 10>{});
  else go(std::integral_constant<int, kMsgChunk>{});
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
  // an edge has one or two sites as children, found by (slot, cluster) in the fused form
  if (e.n > 0 && (e.maxch < 1 || e.maxch > 2 || (e.fp != nullptr && e.ch_rslot == nullptr)))
    return hipErrorInvalidValue;
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

hipError_t launch_set_params(double* h, const double* hfix, const int64_t* pc_hoff, const int64_t* pc_ptr,
                             const int32_t* pc_param, const int64_t* pc_doff, const double* dterm,
                             const int32_t* pc_ncomp, int64_t n_pc, const double* params, hipStream_t s) {
  if (n_pc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_params, dim3(grid_for(n_pc, 256)), dim3(256), 0, s, h, hfix, pc_hoff, pc_ptr, pc_param,
                     pc_doff, dterm, pc_ncomp, n_pc, params);
  return hipGetLastError();
}

hipError_t launch_param_bar(double* out, int accumulate, int64_t n_params, const int64_t* pp_ptr,
                            const int64_t* pp_yoff, const int64_t* pp_doff, const int32_t* pp_D, const double* Y,
                            const double* dterm, bool cplx, hipStream_t s) {
  if (n_params == 0) return hipSuccess;
  hipLaunchKernelGGL(k_param_bar, dim3(grid_for(n_params, 256)), dim3(256), 0, s, out, accumulate, n_params, pp_ptr,
                     pp_yoff, pp_doff, pp_D, Y, dterm, cplx ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adj_pre(const double* a, const double* b, double* btot, double* gbar, double th, double invthL,
                          int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_pre, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, btot, gbar, th, invthL, n);
  return hipGetLastError();
}

hipError_t launch_adj_post(double* a, double* b, const double* btot, const double* etabar, double th, int64_t n,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_post, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, btot, etabar, th, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_extrap(T* dst, const T* nu, const T* ze, double th, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_extrap<T>), dim3(grid_for(n, 256)), dim3(256), 0, s, dst, nu, ze, th, n);
  return hipGetLastError();
}

hipError_t launch_scale_offdiag(double* x, int64_t M, int D, bool cplx, double f, hipStream_t s) {
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_offdiag, dim3(grid_for(M, 256)), dim3(256), 0, s, x, M, D, cplx ? 1 : 0, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_noise(T* x, int64_t n, double scale, uint32_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill_noise<T>), dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, scale, seed);
  return hipGetLastError();
}
template hipError_t launch_fill_noise<float>(float*, int64_t, double, uint32_t, hipStream_t);
template hipError_t launch_fill_noise<double>(double*, int64_t, double, uint32_t, hipStream_t);
template hipError_t launch_extrap<float>(float*, const float*, const float*, double, int64_t, hipStream_t);
template hipError_t launch_extrap<double>(double*, const double*, const double*, double, int64_t, hipStream_t);
template hipError_t launch_cluster<float>(const ClusterArgs<float>&, bool, int, int, int, hipStream_t);
template hipError_t launch_cluster<double>(const ClusterArgs<double>&, bool, int, int, int, hipStream_t);
template hipError_t launch_msg<float>(const MsgArgs<float>&, int, int, hipStream_t);
template hipError_t launch_msg<double>(const MsgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_copy<float>(float*, const float*, int64_t, hipStream_t);
template hipError_t launch_cluster_pair<float>(const ClusterArgs<float>&, const ClusterArgs<float>&, bool, int, int,
                                               hipStream_t);
template hipError_t launch_cluster_pair<double>(const ClusterArgs<double>&, const ClusterArgs<double>&, bool, int,
                                                int, hipStream_t);
template hipError_t launch_copy<double>(double*, const double*, int64_t, hipStream_t);

}  // namespace lrh
