// Internal interface between the host driver (lrh_host.cpp) and the kernels
// (lrh_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lrh {

enum ClusterMode : int {
  MODE_GIBBS = 0,    // F_beta and Gibbs state rho_beta (smoothed dual, Sec. 4.2.2)
  MODE_GROUND = 1,   // lambda_min and normalised ground projector (Sec. 4.2.1)
  MODE_CERTIFY = 2,  // FP64 lambda_min and rounding margin only (no eigenvectors)
};

enum MsgMode : int {
  MSG_GRAD = 0,      // grad[m] = R[child] - T[m]
  MSG_SUBGRAD = 1,   // nu_best copy where improved, then nu += alpha g
  MSG_NESTEROV = 2,  // zeta += g / (theta L); nu = (1 - theta) nu + theta zeta
};

// Packed Hermitian layout: upper-triangle real parts (row-major), then the imaginary
// parts of the strict upper triangle.
__host__ __device__ constexpr int tri_index(int i, int j, int D) {
  return i * D - (i * (i - 1)) / 2 + (j - i);
}
__host__ __device__ constexpr int stri_index(int i, int j, int D) {
  return i * (D - 1) - (i * (i - 1)) / 2 + (j - i - 1);
}
__host__ __device__ constexpr int n_comps(int D, bool cplx) {
  return cplx ? D * D : D * (D + 1) / 2;
}

// Per-iteration scalars of the fused Nesterov loop, read from device memory so that a
// captured graph can be replayed for any stage.
struct FusedParams {
  double theta_prev;   // theta_{k-1}
  double inv_thL_prev; // 1 / (theta_{k-1} L)
  double theta_cur;    // theta_k
  double beta;
  double inv_thL_cur;  // 1 / (theta_k L)
};

template <typename T>
struct ClusterArgs {
  int64_t n;            // clusters in the bucket
  int De, Dc;           // cluster and child dimensions (Dc = 0: no children)
  int maxch, maxpar;
  const int32_t* gid;   // [n] library cluster id
  const int64_t* hoff;  // [n] offset into h (packed comps), -1: h_e = 0
  const int32_t* ch;    // [maxch][n] child-message index in the Dc bucket, -1 unused
  const int32_t* chmask;// [maxch][n] bit mask of the child's sites inside the cluster
  const int32_t* gtab;  // clusters holding a spin-1 site (De not a power of two): [maxch][n][De]
                        // entry i = a(i) | r(i) << 8 | idx(i / NR, i % NR) << 16, with a(i), r(i) the
                        // child and remaining indices of cluster index i and idx(a, r) the inverse
                        // (NR = De / Dc); nullptr for spin-1/2 buckets
  const int32_t* par;   // [maxpar][n] parent-message index in the De bucket, -1 unused
  const int32_t* rslot; // [n] marginal slot in the De marginal buffer, -1: no parents
  const double* h;      // packed term blocks (double)
  // child messages (dimension Dc)
  const T* nu_c; const T* ze_c; int64_t Mc;
  T* Tout;              // partial traces, message layout of the Dc bucket (nullable)
  // parent messages (dimension De)
  const T* nu_p; const T* ze_p; int64_t Mp;
  T* R; int64_t S;      // marginal slots of dimension De (nullable)
  T* marg; const int64_t* marg_off;  // per-cluster marginal output (nullable)
  double* scal;         // per library cluster id: F_beta or lambda_min
  double* scal2;        // per library cluster id: certify margin (MODE_CERTIFY)
  double beta;          // inverse temperature (MODE_GIBBS)
  double theta;         // extrapolation weight when ze_* != nullptr
  double tau_rel;       // ground-space threshold (MODE_GROUND)
  const FusedParams* tab;  // device table row: theta (extrapolation) and beta replace the
                           // fields above (graph-replayed plain iterations); nullptr: unused
  int max_sweeps;
  double tol;           // relative off-diagonal tolerance
  unsigned long long* noconv;
  unsigned long long* nonfinite;
  // ---- fused update of the previous iteration (register kernel only) ----
  const FusedParams* fp;      // device pointer, nullptr: no fused update
  const T* nu_c_prev; const T* ze_c_prev; const T* Tprev_c; const T* Rprev_c;
  const int32_t* rslot_of_msg_c; int64_t Sc;
  const int32_t* ch_rslot;    // [maxch][n] child's marginal slot by (slot, cluster): read beside ch
  T* nu_c_new; T* ze_c_new;   // written by the parent (this cluster)
  const T* nu_p_prev; const T* ze_p_prev; const T* Tprev_p; const T* Rprev_p;
  int fused_first;            // 1: iteration 0 of a call, state already current
  // ---- adjoint (k_cluster_vjp) ----
  const T* gb_c; const T* gb_p;  // gradient cotangent gbar, child / parent buckets (nullable)
  double gb_offscale;            // scale of off-diagonal gbar elements (1, or 1/2 for packed coords)
  const double* qbar;            // [n_inst] cotangent of Q per instance (nullable: 0)
  const int32_t* cinst;          // [n_clusters] instance of every library cluster
  // ---- large clusters (De >= 128): per-workgroup scratch slab in device memory ----
  void* big_scratch;             // big_blocks slabs of big_slab elements of T
  int64_t big_slab;
  int64_t big_blocks;
  // ---- workgroup scaling-and-squaring Gibbs kernel, De >= 32: per-workgroup FP64 slab ----
  double* expm_scratch;          // expm_blocks slabs of expm_slab doubles
  int64_t expm_slab;
  int64_t expm_blocks;
  // ---- certification at De = 16, 32: tridiagonals of the bucket (2 De n doubles); nullptr: the
  // one-wave kernel with multisection instead ----
  double* cert_ws;
  // ---- certification at De >= 64: 0 Lanczos + Cholesky certificate at De = 256 (tridiagonalisation
  // where the certificate fails, and at De = 64, 128), 1 tridiagonalisation only, 2 test hook: the
  // certificate is tried at a shift above lambda_min at every De >= 64, so every such cluster takes
  // the tridiagonalisation, 3 the certificate at every De >= 64 ----
  int cert_method;
  unsigned long long* cert_fallback;   // clusters certified by the tridiagonalisation instead
};

template <typename T>
struct MsgArgs {
  int64_t M, comps, S;
  const int32_t* rslot;   // [M] child's marginal slot
  const int32_t* inst;    // [M] instance
  const T* R; const T* Tm;
  T* nu; T* ze; T* nu_best; T* grad;
  const T* nu_src; const T* ze_src;  // state read from here (nullptr: nu / ze, in place)
  const int32_t* improved;  // [n_inst] (subgradient best tracking)
  double alpha, theta, inv_thL;
  const FusedParams* fp;    // if set, theta/inv_thL come from here (theta_prev, or theta_cur
  int fp_cur;               // when fp_cur is set)
};

// ---- launchers (lrh_kernels.hip) ----
// block: threads per block of the register kernels; W: lanes per cluster of the LDS kernels
// (64/W clusters per wave), one of the shapes listed by lds_shapes()
template <typename T>
hipError_t launch_cluster(const ClusterArgs<T>& a, bool cplx, int mode, int block, int W, hipStream_t s);
// lanes-per-cluster shapes compiled for an LDS bucket of dimension De (returns the count)
int lds_shapes(int De, int* out);
// every launch shape available for a bucket in a given precision / field / mode, best guess
// first: 1 = one lane per cluster (register kernel), otherwise lanes per cluster of the LDS kernel
int cluster_shapes(int De, int Dc, bool dbl, bool cplx, int mode, int* out);
template <typename T>
hipError_t launch_msg(const MsgArgs<T>& a, int mode, int block, hipStream_t s);
hipError_t launch_reduce(const double* scal, const int64_t* inst_ptr, int64_t n_inst, double* out,
                         const double* scal2, double* out2, double* q_best, int32_t* improved,
                         double* q_hist, hipStream_t s);
constexpr int kFusedTableMax = 65;
constexpr int kTableRows = 65;  // rows of the device parameter table (chunk of 64 + 1)
struct FusedTable { FusedParams p[kFusedTableMax]; };
hipError_t launch_set_fused(FusedParams* dst, const FusedTable& v, int n, hipStream_t s);
hipError_t launch_widen(double* dst, const float* src, int64_t n, hipStream_t s);
// two-bucket fused/plain launch for 2-local problems: edges (De=4, Dc=2) and sites (De=2)
template <typename T>
hipError_t launch_cluster_pair(const ClusterArgs<T>& edges, const ClusterArgs<T>& sites, bool cplx,
                               int mode, int block, hipStream_t s);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, int64_t n, hipStream_t s);

// ---- adjoint helpers ----
hipError_t launch_cluster_vjp(const ClusterArgs<double>& a, bool cplx, int mode, hipStream_t s);
// h_e = hfix_e + sum_t params[p_t] * dterm_t for the clusters listed in (pc_gid... CSR)
hipError_t launch_set_params(double* h, const double* hfix, const int64_t* pc_hoff, const int64_t* pc_ptr,
                             const int32_t* pc_param, const int64_t* pc_doff, const double* dterm,
                             const int32_t* pc_ncomp, int64_t n_pc, const double* params, hipStream_t s);
// param_bar[p] (+)= sum over the parameter's terms of <Y_e, dterm_t> (Y per cluster, packed)
hipError_t launch_param_bar(double* out, int accumulate, int64_t n_params, const int64_t* pp_ptr,
                            const int64_t* pp_yoff, const int64_t* pp_doff, const int32_t* pp_D, const double* Y,
                            const double* dterm, bool cplx, hipStream_t s);
// reverse Nesterov step on message vectors (length n)
hipError_t launch_adj_pre(const double* a, const double* b, double* btot, double* gbar, double th, double invthL,
                          int64_t n, hipStream_t s);
hipError_t launch_adj_post(double* a, double* b, const double* btot, const double* etabar, double th, int64_t n,
                           hipStream_t s);
// x[i] = scale * (uniform(-1, 1) from a 64-bit mix of (seed, i))
template <typename T>
hipError_t launch_fill_noise(T* x, int64_t n, double scale, uint32_t seed, hipStream_t s);
template <typename T>
hipError_t launch_extrap(T* dst, const T* nu, const T* ze, double th, int64_t n, hipStream_t s);
// sustained FP64 matrix-core rate probe: blocks x 256 threads, 8 MFMA chains of `iters` steps per
// lane; out: blocks * 256 doubles
hipError_t launch_mfma_f64_rate(double* out, int blocks, int iters, hipStream_t s);
// scale the off-diagonal components of every message of a bucket by f
hipError_t launch_scale_offdiag(double* x, int64_t M, int D, bool cplx, double f, hipStream_t s);

}  // namespace lrh
