/*
 * lrh.h -- C ABI of the local-relaxation message-passing library for MI355X (gfx950).
 *
 * The library solves the partial-Lagrangian dual of the cluster-consistent
 * relaxation f*_C of a local Hamiltonian H = sum_e h_e (paper: Sec. 3.2, definition
 * of the cluster-consistent set and eq. cluster_relaxation_energy; Sec. 4, dual
 * Q_C(nu) = sum_e lambda_min(theta_e(nu)) and its smoothed form Q_{C,beta}).
 *
 * Conventions shared by every call
 *   - Every call returns an lrh_status; nothing throws across the ABI.  On failure
 *     lrh_last_error() returns a thread-local message.
 *   - "host" pointers are read during the call only; the caller keeps ownership.
 *     "device" pointers are HIP device memory owned by the caller; the call
 *     enqueues work on `stream` and returns without waiting: results are valid once
 *     the stream is synchronised.
 *   - Sites are spin-1/2 (d = 2) or spin-1 (d = 3).  Clusters of spin-1/2 sites hold at most 8
 *     sites (D_e <= 256); a cluster holding a spin-1 site has D_e = prod d <= 64.  A cluster's
 *     basis is the big-endian mixed-radix product basis of its sites in ascending order (first
 *     site most significant), so A_{s0} (x) B_{s1} = kron(A, B).
 *   - Message layout (structure of arrays).  Messages nu_{e->f} (e a cluster, f one of
 *     its covering children) are grouped into buckets by D_f.  Bucket b holds M_b
 *     messages of C_b components each; component c of message m lives at element
 *     offset_b + c * M_b + m.  For a real problem (all terms real, LRH_REAL) the
 *     components are the upper triangle A[i][j], i <= j, in row-major order
 *     (C_b = D(D+1)/2).  For a complex problem they are the real parts of the upper
 *     triangle in the same order, followed by the imaginary parts of the strict upper
 *     triangle (C_b = D^2).  Element type is double, or float when the call's flags
 *     carry LRH_F32.  lrh_query() reports every bucket; lrh_export_messages() reports
 *     which cluster pair each message belongs to.
 *   - Instances: sites carry an instance id; clusters never span instances and every
 *     per-instance output is indexed by that id.
 */
#ifndef LRH_H
#define LRH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LRH_OK = 0,
  LRH_E_INVALID = 1,      /* bad argument: non-Hermitian term, cluster spanning instances,
                             beta <= 0, Lipschitz <= 0, null required pointer, ...          */
  LRH_E_UNSUPPORTED = 2,  /* D_e > 256 (> 64 with a spin-1 site), site dimension not 2 or 3,
                             children of one cluster with different dimensions              */
  LRH_E_NOMEM = 3,        /* device or host allocation failed                             */
  LRH_E_DEVICE = 4,       /* a HIP runtime call failed                                    */
  LRH_E_NOCONV = 5,       /* a Jacobi eigen-solve hit its sweep cap (see lrh_check)       */
  LRH_E_NONFINITE = 6     /* NaN / Inf found in a state or a bound (see lrh_check)        */
} lrh_status;

/* flags for lrh_problem_desc.flags */
#define LRH_SUBINTERVALS 0x1u  /* add every contiguous run of each top cluster (Y_t, eq.
                                  interval_set_defn: intervals "with their subsets")      */
#define LRH_TWO_LEVEL    0x2u  /* two-level family: the top clusters and the intersections of
                                  two top clusters that no other such intersection strictly
                                  contains, nothing else (no term supports, no singletons).
                                  Each term is split evenly over the top clusters holding its
                                  support (LRH_E_INVALID if none does).  On a chain with the
                                  windows of length t as tops this keeps Y_t's optimum with
                                  only the windows and their overlaps (Sec. 3.2, Sec. 4.2).
                                  Excludes LRH_SUBINTERVALS.                               */

/* flags for the compute calls */
#define LRH_F32    0x1u   /* state buffers (nu, zeta, grad, marginals) are float, and the
                             iterations compute in FP32; certification stays FP64.  Gibbs
                             states of clusters with D_e >= 16 come from scaling and
                             squaring: a degree-8 Taylor polynomial and the first four
                             squarings in FP64, the later squarings in FP32 (FP64 messages:
                             degree 12, every squaring in FP64); the result is within the
                             float rounding of the messages                                 */
#define LRH_FUSED  0x2u   /* graph-replayed iterations: for 2-local problems one launch per
                             iteration (the message update of the previous step folded into
                             the cluster kernel); otherwise the plain launches of each
                             iteration, driven by a device table of per-iteration scalars.
                             Either form is captured once per 64-iteration chunk            */
#define LRH_PACKED_COTANGENT 0x4u  /* message cotangents (gbar in, nu_bar out) are taken with
                             respect to the packed storage components instead of the
                             Frobenius inner product of the Hermitian matrices (they differ by
                             a factor 2 on off-diagonal components)                        */

typedef struct lrh_problem_s* lrh_problem;   /* opaque; owned by the library */

/* Problem description (all HOST memory, copied during lrh_build_clusters).
 * H = sum_t h_t, term t acting on sites term_sites[term_ptr[t] .. term_ptr[t+1]) given
 * in ascending order; its dense row-major block starts at term_off[t] in term_re /
 * term_im (term_im == NULL: every term is real, the problem is solved in real
 * arithmetic).  The cluster family (Sec. 3.2) is the list of top clusters
 * top_sites[top_ptr[c] .. top_ptr[c+1]) (ascending); the library adds every term
 * support and every singleton, plus contiguous runs when LRH_SUBINTERVALS is set
 * (LRH_TWO_LEVEL: only the maximal pairwise overlaps of the tops), and keeps the
 * covering relations of the inclusion poset (Sec. 4.2: constraints between consecutive
 * poset levels suffice).  site_instance may be NULL (one instance). */
typedef struct {
  int32_t n_sites;
  const int32_t* site_dim;        /* [n_sites], 2 or 3                                   */
  int32_t n_terms;
  const int64_t* term_ptr;        /* [n_terms+1]                                         */
  const int32_t* term_sites;
  const int64_t* term_off;        /* [n_terms+1], offsets into term_re / term_im         */
  const double* term_re;
  const double* term_im;          /* NULL => real problem                                */
  int32_t n_top;
  const int64_t* top_ptr;         /* [n_top+1]                                           */
  const int32_t* top_sites;
  const int32_t* site_instance;   /* [n_sites] or NULL                                   */
  uint32_t flags;                 /* LRH_SUBINTERVALS or LRH_TWO_LEVEL                   */
  /* Optional linear parametrisation of terms (for gradients with respect to couplings):
   * term t with term_param[t] = p >= 0 is h_t(c) = h_t + (c_p - params[p]) * dterm_t, with
   * dterm_t = d h_t / d c_p stored like the terms (term_off, dterm_im NULL for a real
   * problem).  n_params = 0 and NULL pointers: no parameters. */
  int32_t n_params;
  const int32_t* term_param;      /* [n_terms], -1: constant term                       */
  const double* dterm_re;
  const double* dterm_im;
  const double* params;           /* [n_params] values the term blocks were given at    */
} lrh_problem_desc;

#define LRH_MAX_BUCKETS 8
typedef struct {
  int64_t n_clusters, n_msgs, n_instances;
  int32_t is_real;
  int32_t max_D;
  int32_t n_buckets;                       /* message buckets, by D_f ascending        */
  int32_t bucket_D[LRH_MAX_BUCKETS];
  int64_t bucket_count[LRH_MAX_BUCKETS];   /* M_b                                       */
  int64_t bucket_comps[LRH_MAX_BUCKETS];   /* C_b                                       */
  int64_t bucket_offset[LRH_MAX_BUCKETS];  /* element offset of bucket b               */
  int64_t nu_len;                          /* elements of one message vector           */
  int64_t marg_len;                        /* elements of the per-cluster marginal
                                              buffer of lrh_dual_eval (packed like a
                                              message of size D_e, clusters in the
                                              order of lrh_export_clusters)            */
  double Lambda_G;                         /* Lipschitz factor: L = beta * Lambda_G / 2 */
  double Gamma_G;                          /* sum_e log D_e (smoothing-error lemma)     */
  int32_t max_sweeps;                      /* Jacobi sweep cap in use                   */
  int32_t n_params;                        /* parameters of the term parametrisation    */
} lrh_layout;

/* Build the cluster poset, message layout and device-resident problem data on HIP
 * device `hip_device` (a0: poset + layouts; Sec. 3.2, Sec. 4.2).  hip_device < 0 builds
 * the poset and layout on the host only (lrh_query / lrh_export_* work, every compute
 * call returns LRH_E_INVALID).
 * Errors: LRH_E_INVALID (non-Hermitian term beyond 1e-12 * max|h|, site out of range,
 * unsorted or repeated sites, cluster spanning instances), LRH_E_UNSUPPORTED (site
 * dimension not 2 or 3, a cluster with more than 8 sites or, holding a spin-1 site, with
 * D_e > 64, a cluster whose children have different dimensions), LRH_E_NOMEM, LRH_E_DEVICE.  On success *out owns device
 * memory until lrh_destroy. */
lrh_status lrh_build_clusters(const lrh_problem_desc* desc, int hip_device, lrh_problem* out);

/* Sizes and layout of a built problem (host struct filled in). */
lrh_status lrh_query(lrh_problem p, lrh_layout* out);

/* Host copies of the poset.  Clusters are numbered in the library's order (grouped by
 * instance); cluster c has sites sites[ptr[c] .. ptr[c+1]).  ptr: [n_clusters+1],
 * sites: [ptr[n_clusters]], instance: [n_clusters] (any of them may be NULL). */
lrh_status lrh_export_clusters(lrh_problem p, int64_t* ptr, int32_t* sites, int32_t* instance);

/* For every message, in bucket order (bucket 0 first, then by index within the bucket):
 * parent and child cluster ids, bucket and index within the bucket.  Arrays of length
 * n_msgs; any may be NULL. */
lrh_status lrh_export_messages(lrh_problem p, int32_t* parent, int32_t* child,
                               int32_t* bucket, int64_t* index);

/* Dual value and (sub)gradient at nu (Sec. 4.1 / 4.2).
 *   beta > 0 : q_dev[i] = Q_{C,beta}(nu) of instance i = sum_e F_beta(theta_e), and
 *              grad = rho_f - Tr_{e\f} rho_e (Gibbs states; Sec. 4.2.2);
 *   beta == 0: q_dev[i] = Q_C(nu) = sum_e lambda_min(theta_e) and grad = mu_f - Tr mu_e
 *              with mu the normalised ground-space projector (Sec. 4.2.1).
 * nu: device, nu_len elements (LRH_F32: float).  q_dev: device double[n_instances].
 * grad_dev: device, nu_len elements of nu's type, or NULL.  marg_dev: device, marg_len
 * elements of nu's type receiving every cluster's rho_e / mu_e, or NULL.
 * Errors: LRH_E_INVALID (null nu or q_dev, beta < 0), LRH_E_DEVICE. */
lrh_status lrh_dual_eval(lrh_problem p, const void* nu, uint32_t flags, double beta,
                         double* q_dev, void* grad_dev, void* marg_dev, hipStream_t stream);

/* Algorithm 1 (subgradient ascent), n_iter iterations k = k0 .. k0+n_iter-1 with step
 * alpha_k = step_scale / sqrt(k + 1) when step_kind == 0, or the constant step_scale
 * when step_kind == 1.  At each k: q^k = Q(nu^k) per instance; where q^k > q_best the
 * instance's messages are copied to nu_best and q_best updated; then
 * nu <- nu + alpha_k (mu_f - Tr_{e\f} mu_e).  nu, nu_best: device, nu_len elements
 * (LRH_F32: float); q_best_dev: device double[n_instances], initialise to -inf before
 * the first call.  q_hist_dev: device double[n_iter * n_instances] (row k - k0) or NULL.
 * Errors: LRH_E_INVALID (null pointers, n_iter < 0, k0 < 0, step_scale <= 0). */
lrh_status lrh_step_subgrad(lrh_problem p, void* nu, void* nu_best, double* q_best_dev,
                            int64_t k0, int32_t n_iter, int32_t step_kind, double step_scale,
                            double* q_hist_dev, uint32_t flags, hipStream_t stream);

/* State of Algorithm 2 within one smoothing stage. */
typedef struct {
  int64_t k;        /* iterations done in this stage; k == 0 starts a stage: zeta <- nu,
                       theta <- 1 (for nu = 0 this is Algorithm 2's initialisation)      */
  double theta;     /* theta_k (updated by the call)                                     */
  double beta;      /* inverse temperature of the stage (> 0)                            */
  double L;         /* Lipschitz bound L_beta (> 0); 0 selects the paper's beta Lambda_G / 2
                       (Sec. 4.2.2; Delta_G + d for 2-local families, Sec. 4.1.2), written back */
} lrh_nesterov_state;

/* Algorithm 2 (accelerated ascent on the smoothed dual): n_iter iterations of
 *   eta = (1 - theta_k) nu + theta_k zeta;  g = grad Q_beta(eta);
 *   zeta += g / (theta_k L);  nu = (1 - theta_k) nu + theta_k zeta;
 *   theta_{k+1} = (sqrt(theta_k^4 + 4 theta_k^2) - theta_k^2) / 2.
 * nu, zeta: device, nu_len elements (LRH_F32: float).  st: host, updated on return.
 * With LRH_FUSED the iterations run as one launch each from a captured graph; the
 * result is the same arithmetic in a different launch structure.
 * Errors: LRH_E_INVALID (null pointers, beta <= 0 or not finite, L < 0, n_iter < 0). */
lrh_status lrh_step_nesterov(lrh_problem p, void* nu, void* zeta, lrh_nesterov_state* st,
                             int32_t n_iter, uint32_t flags, hipStream_t stream);

/* Certified lower bound (weak duality, Sec. 4.1): FP64 lambda_min of every cluster at
 * nu, summed per instance in a fixed order.  q_dev[i] = Q_C(nu), margin_dev[i] = sum_e m_e,
 * the rounding margin of each cluster's FP64 solve; the certified bound is
 * q - margin <= f*_C <= E0.  By dimension:
 *   D_e <= 8 (Jacobi): m_e = 8 D_e eps_64 ||theta_e||_F + r_e, r_e the Frobenius norm of the
 *     off-diagonal part left by the sweeps (the bound holds even when a solve stops at its
 *     sweep cap);
 *   D_e = 16, 32 (Householder tridiagonalisation, Sturm bisection): m_e = 8 D_e eps_64
 *     ||theta_e||_F, the value being the lower end of the Sturm bracket;
 *   D_e = 64, 128: as D_e = 16, 32 (one workgroup per cluster, the matrix in a device slab);
 *   D_e = 256 (lambda_min only, Sec. 4.2: Lanczos for the Ritz value rho, then one
 *     Cholesky factorisation of theta_e - sigma I, sigma = rho - eta, that proves
 *     lambda_min >= sigma - g || |R| ||_1 || |R| ||_inf - 2 u max_i |theta_ii - sigma| - a_e,
 *     g the Cholesky backward-error constant, a_e an assembly-rounding term): the value is rho
 *     and m_e = rho minus that bound.  Where the factorisation breaks down the cluster is
 *     certified by the tridiagonalisation instead (counted, see lrh_certify_fallbacks).
 * lrh_set_certify_method selects the tridiagonalisation, or the certificate, at every D_e >= 64.
 * Certification always uses the FP64 default Jacobi tolerance (lrh_set_jacobi's tolerance
 * does not apply; its sweep cap does).  nu may be float (LRH_F32); it is widened to double
 * before theta_e is formed.  lmin_dev: device double[n_clusters] (library cluster order) or NULL.
 * Errors: LRH_E_INVALID (null nu/q/margin). */
lrh_status lrh_certify(lrh_problem p, const void* nu, uint32_t flags, double* q_dev,
                       double* margin_dev, double* lmin_dev, hipStream_t stream);

/* lrh_certify for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and results, but the
 * call allocates nothing.  Its workspace -- the FP64 copy of float messages (LRH_F32) and one
 * matrix slab per workgroup of the tridiagonalisation kernel at D_e >= 64 -- is a fixed 64 MiB
 * array in device memory that the library holds on every GPU it runs on until the process ends.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Nothing in the array needs to start
 * at zero.  With fewer slabs than clusters each workgroup certifies several clusters in turn.
 * The problem itself (its terms, index tables and per-cluster values) is the one allocated by
 * lrh_build_clusters; outputs as in lrh_certify.
 * Errors: LRH_E_INVALID (null nu/q/margin, host-only problem), LRH_E_UNSUPPORTED (LRH_F32 with
 * nu_len * 8 bytes above 64 MiB), LRH_E_DEVICE (the array's device address could not be found
 * when the first problem was built on this GPU, or a launch failed). */
lrh_status lrh_certify_noalloc(lrh_problem p, const void* nu, uint32_t flags, double* q_dev,
                               double* margin_dev, double* lmin_dev, hipStream_t stream);

/* Move the parametrised terms to new parameter values (device double[n_params]):
 * h_e = sum of the constant terms + sum_t params[p_t] * dterm_t, recomputed on the device.
 * Errors: LRH_E_INVALID (no parameters, null pointer). */
lrh_status lrh_set_params(lrh_problem p, const double* params_dev, hipStream_t stream);

/* Adjoint of lrh_dual_eval (FP64): cotangents qbar (device double[n_instances], NULL = 0) of
 * the per-instance dual values and gbar (device, nu_len doubles, NULL = 0) of the gradient
 * are pulled back to the messages and to the parameters:
 *   Y_e = qbar rho_e + D rho_e[(B gbar)_e],  nu_bar = B^* Y = Y_f - Tr_{e\f} Y_e,
 *   param_bar[p] = sum over the parameter's terms of <Y_e, dterm_t>,
 * with B the linear map from messages to augmented Hamiltonians (grad Q_beta = B^* rho,
 * Sec. 4.1.2 / Lipschitz lemma) and D rho the Daleckii-Krein derivative of the Gibbs state.
 * beta == 0 differentiates Q itself with the ground projector (gbar must be NULL).
 * nu_bar_dev: device, nu_len doubles (or NULL); param_bar_dev: device double[n_params] or NULL.
 * flags: LRH_PACKED_COTANGENT; LRH_F32 is not supported (LRH_E_UNSUPPORTED), nor complex
 * clusters with D_e = 64, nor any cluster with D_e > 64.
 * Errors: LRH_E_INVALID (null nu, beta < 0, gbar with beta == 0). */
lrh_status lrh_dual_vjp(lrh_problem p, const void* nu, uint32_t flags, double beta, const double* qbar_dev,
                        const void* gbar_dev, void* nu_bar_dev, double* param_bar_dev, hipStream_t stream);

/* Certified value after T accelerated steps and its gradient (FP64):
 *   B_T = Q(nu^T) per instance, nu^T = T steps of Algorithm 2 at fixed beta and Lipschitz L
 *   (L = 0: beta Lambda_G / 2) from nu0 (zeta0 = nu0, theta0 = 1; nu0 == NULL: zero messages),
 * and the reverse-mode derivative of sum_i qbar_i B_T,i (qbar NULL: all ones) with respect to
 * the parameters (param_bar_dev, double[n_params]) and to nu0 (nu0_bar_dev, nu_len doubles,
 * LRH_PACKED_COTANGENT applies).  The forward pass keeps every extrapolated point (T * nu_len
 * doubles of workspace); each reverse step is one lrh_dual_vjp at that point.  The rounding
 * margin of lrh_certify is not included in B_T.
 * Errors: LRH_E_INVALID (beta <= 0, L < 0, T < 0, null bound_dev), LRH_E_UNSUPPORTED as for
 * lrh_dual_vjp. */
lrh_status lrh_unrolled_bound_grad(lrh_problem p, const double* nu0_dev, double beta, double L, int32_t T,
                                   const double* qbar_dev, double* bound_dev, double* param_bar_dev,
                                   double* nu0_bar_dev, uint32_t flags, hipStream_t stream);

/* Synchronise `stream` and report the eigen-solver health flags accumulated since the
 * last lrh_check: *noconv = clusters that hit the sweep cap, *nonfinite = clusters with
 * a NaN/Inf eigenvalue.  Returns LRH_E_NONFINITE or LRH_E_NOCONV when either is
 * non-zero (NONFINITE first), LRH_OK otherwise.  Either pointer may be NULL. */
lrh_status lrh_check(lrh_problem p, hipStream_t stream, int64_t* noconv, int64_t* nonfinite);

/* Synchronise `stream`, then *count = clusters of D_e >= 64 whose Cholesky certificate broke
 * down since the last call (certified by the tridiagonalisation instead), and reset it.
 * Errors: LRH_E_INVALID (null problem or count, host-only problem). */
lrh_status lrh_certify_fallbacks(lrh_problem p, hipStream_t stream, int64_t* count);

/* Certification of D_e >= 64 clusters: method 0 (default) the Lanczos + Cholesky certificate at
 * D_e = 256 and Householder tridiagonalisation + Sturm bisection at D_e = 64, 128; 1 the
 * tridiagonalisation at every D_e >= 64; 3 the certificate at every D_e >= 64; 2 (for tests of
 * the fallback) the certificate at every D_e >= 64, tried at a shift above lambda_min, so it breaks
 * down and every such cluster is certified by the tridiagonalisation.
 * Errors: LRH_E_INVALID (null problem, other method). */
lrh_status lrh_set_certify_method(lrh_problem p, int32_t method);

/* Launch shapes (the W of the calls below), per cluster bucket and precision:
 *   W = 1      register kernel, one lane per cluster (D_e <= 8), Jacobi
 *   W = 8..64  LDS kernel, W lanes per cluster, 64/W clusters per wave (8 <= D_e <= 64), Jacobi
 *   W = 1024   one 1024-thread workgroup per cluster, matrix in a device slab (D_e = 128, 256),
 *              Jacobi; ground projector only once the exponential exists for the bucket
 *   W = 0      Gibbs state exp(-beta theta)/Z by scaling and squaring on the FP64 matrix cores,
 *              no eigenvectors, one wave per cluster, matrices in registers (D_e = 16, 32;
 *              Gibbs passes only, the default there)
 *   W = 4      the same on one 256-thread workgroup per cluster, matrices in a device slab
 *              (D_e >= 32; the default for D_e >= 64)
 *   W = 5      clusters holding a spin-1 site (D_e not a power of two): the LDS Jacobi kernel
 *              driven by index tables (lift and partial-trace maps per cluster and child) on the
 *              next power of two, with decoupled padding; every mode, the only shape there
 * Certification at D_e >= 16 (spin-1/2) uses its own kernels (W = 2 internally): at D_e = 16
 * and 32 Householder tridiagonalisation with one lane group per cluster holding the rows in
 * registers, then Sturm bisection with one lane per cluster; at D_e >= 64 one workgroup per
 * cluster runs the tridiagonalisation (64, 128) or Lanczos and the Cholesky certificate (256; see
 * lrh_certify);
 * the ground projector and the adjoint use the Jacobi shapes.  The adjoint (lrh_dual_vjp,
 * lrh_unrolled_bound_grad) covers spin-1/2 clusters only.
 *
 * Launch-shape autotuner (form 2): for every cluster bucket, time the Gibbs pass of the
 * candidate shapes -- threads per block {64, 128, 256} for the register kernels (D_e <= 4),
 * the compiled W above otherwise; the slab Jacobi is not timed where the exponential exists --
 * on seeded random messages, in the precision of `flags` (LRH_F32 or FP64), and keep the
 * fastest.  cache_path (may be NULL) names a JSON file of earlier choices keyed by (D_e,
 * D_child, real/complex, precision, bucket size): cached buckets are not re-measured, and the
 * file is rewritten with every choice.  Synchronous.  Every shape computes the same quantities;
 * results agree to rounding. */
lrh_status lrh_autotune(lrh_problem p, uint32_t flags, const char* cache_path, hipStream_t stream);

/* Launch shapes in use, one entry per cluster bucket (at most `cap` written; *count = number
 * of buckets): dimensions, cluster count, block / lanes-per-cluster, measured microseconds
 * (0 when not measured).  Host arrays, any may be NULL except count. */
lrh_status lrh_get_shapes(lrh_problem p, int32_t cap, int32_t* De, int32_t* Dc, int64_t* n, int32_t* block,
                          int32_t* W, double* us, int32_t* count);

/* Force the launch shape of every cluster bucket of dimension De for the precision of `flags`
 * (LRH_F32: FP32 iterations, else FP64): block = threads per block of the register kernel
 * (64, 128, 256), W one of the shapes listed above for the Gibbs pass.  Errors:
 * LRH_E_INVALID (no such bucket, bad block), LRH_E_UNSUPPORTED (shape not compiled for that
 * bucket). */
lrh_status lrh_set_shape(lrh_problem p, int32_t De, int32_t block, int32_t W, uint32_t flags);

/* Per-bucket kernel timing for roofline accounting: runs reps + 1 launches of every cluster
 * bucket's kernel (Gibbs state at beta > 0, ground projector at beta = 0) at the messages nu
 * (device, precision of `flags`), in each bucket's current shape, on `stream`, and writes the
 * average duration of one launch in microseconds to us[b] (host array, one entry per bucket in
 * lrh_get_shapes order).  Overwrites the library's workspace; synchronises the stream.
 * Errors: LRH_E_INVALID (null pointer, reps < 1, beta < 0), LRH_E_DEVICE. */
lrh_status lrh_time_buckets(lrh_problem p, const void* nu, uint32_t flags, double beta, int32_t reps, double* us,
                            hipStream_t stream);

/* Per-bucket timing of the accelerated message update (a6: zeta += g / (theta L), nu averaged;
 * Algorithm 2) for roofline accounting: one Gibbs pass at beta > 0 on nu fills the workspace,
 * then reps + 1 launches of every message bucket's update run on nu and zeta in place (device,
 * nu_len elements each, precision of `flags`; both are overwritten, pass scratch copies), and
 * the average duration of one launch in microseconds goes to us[b] (host array, one entry per
 * message bucket in lrh_query order).  Overwrites the library's workspace; synchronises the
 * stream.  Errors: LRH_E_INVALID (null pointer, reps < 1, beta <= 0), LRH_E_DEVICE. */
lrh_status lrh_time_messages(lrh_problem p, void* nu, void* zeta, uint32_t flags, double beta, int32_t reps,
                             double* us, hipStream_t stream);

/* Jacobi sweep cap (default 30) and relative off-diagonal tolerance (0 = default:
 * 4 eps of the iteration precision).  Like lrh_set_shape, lrh_autotune and lrh_set_slab_limit,
 * this drops the graphs captured for LRH_FUSED (they hold the old settings); it waits for the
 * device to finish with them first. */
lrh_status lrh_set_jacobi(lrh_problem p, int32_t max_sweeps, double rel_tol);

/* Cap the number of per-workgroup FP64 scratch slabs of the large-cluster kernels (workgroup
 * Gibbs kernel and tridiagonal certification at D_e >= 32, slab Jacobi at D_e >= 128): a slab
 * holds up to five D_e x D_e matrices (complex D_e = 256: 5.2 MB), and by default up to 1024
 * (512 at D_e = 256) are allocated.  With fewer slabs than clusters each workgroup processes
 * several clusters in turn in its slab; results do not depend on the cap.  max_slabs = 0
 * restores the default.  Memory already allocated is kept, only its first max_slabs slabs are
 * used.  Errors: LRH_E_INVALID (null problem, max_slabs < 0). */
lrh_status lrh_set_slab_limit(lrh_problem p, int64_t max_slabs);

/* Measurement aid for roofline reports: the FP64 matrix-core rate this device sustains (TFLOP/s),
 * from eight independent chains of v_mfma_f64_16x16x4_f64 per lane at eight waves per SIMD on
 * every compute unit, timed with events on `stream` (synchronous; allocates and frees its own
 * small output buffer).  The published dense FP64 peak is the nominal figure; this is what the
 * instruction delivers at the device's operating clocks.
 * Errors: LRH_E_INVALID (null tflops), LRH_E_DEVICE. */
lrh_status lrh_measure_fp64_mfma(int hip_device, double* tflops, hipStream_t stream);

void lrh_destroy(lrh_problem p);
const char* lrh_last_error(void);
/* Static text naming the HIP headers the library was compiled against and its device
 * architecture (the runtime serving the process may be another release of the same major). */
const char* lrh_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* LRH_H */
