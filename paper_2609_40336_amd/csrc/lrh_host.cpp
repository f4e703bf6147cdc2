// Host side of the library: problem validation, the cluster poset, device layouts, and
// the drivers of Algorithm 1 (subgradient) and Algorithm 2 (accelerated smoothed ascent).
//
// Poset (paper Sec. 3.2 and Sec. 4.2): C_full holds the top clusters, every term support,
// every singleton and, for the interval hierarchy, every contiguous run of a top
// cluster; only covering relations (maximal proper subsets present in C_full) carry
// messages.  Terms are added to the cluster equal to their support.  The two-level family
// holds only the top clusters and their maximal pairwise overlaps; each term is then split
// evenly over the top clusters that hold its support.
#include <hip/hip_runtime.h>
#include <hip/hip_version.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "lrh.h"
#include "lrh_internal.h"

using namespace lrh;

namespace {

thread_local std::string g_err;

lrh_status fail(lrh_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e__ = (expr);                                                                \
    if (e__ != hipSuccess)                                                                  \
      return fail(LRH_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e__));        \
  } while (0)

constexpr int kMaxSites = 8;  // D_e <= 256 for spin-1/2 sites
constexpr int kMaxGenericD = 64;  // clusters holding a spin-1 site: D_e <= 64 (table-driven kernel)

// Clusters whose dimension is not a power of two hold a spin-1 (d = 3) site; their buckets use the
// table-driven kernels (index maps instead of site bit masks).
inline bool generic_dim(int D) { return (D & (D - 1)) != 0; }

struct Key {
  int k = 0;
  int32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool operator==(const Key& o) const {
    if (k != o.k) return false;
    for (int i = 0; i < k; ++i)
      if (s[i] != o.s[i]) return false;
    return true;
  }
};
struct KeyHash {
  size_t operator()(const Key& key) const {
    uint64_t h = 1469598103934665603ull ^ (uint64_t)key.k;
    for (int i = 0; i < key.k; ++i) {
      h ^= (uint64_t)(uint32_t)key.s[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

struct CBucket {
  int De = 0, Dc = 0, maxch = 0, maxpar = 0;
  int block = 64;     // threads per block (register kernels)
  int W = 64;         // FP32 iterations: lanes per cluster (1 = register kernel, else LDS kernel)
  int W64 = 64;       // FP64 iterations
  double tuned_us = 0.0;
  int64_t n = 0;
  int mb_child = -1;  // message bucket of the children (dimension Dc)
  int mb_self = -1;   // message bucket of dimension De (messages received from parents)
  std::vector<int32_t> h_gid;
  int32_t* gid = nullptr;
  int64_t* hoff = nullptr;
  int32_t* ch = nullptr;
  int32_t* chmask = nullptr;
  int32_t* par = nullptr;
  int32_t* rslot = nullptr;
  int32_t* chrs = nullptr;   // [maxch][n] marginal slot of each child (-1: none)
  int32_t* gtab = nullptr;   // clusters with a spin-1 site: [maxch][n][De] index maps (see ClusterArgs)
};

struct MBucket {
  int D = 0;
  int64_t M = 0, comps = 0, offset = 0;  // message layout
  int64_t S = 0, comps_r = 0, roff = 0;  // marginal slots (clusters of dim D with parents)
  int32_t* rslot = nullptr;              // [M] child's marginal slot
  int32_t* inst = nullptr;               // [M] instance of the message
};

template <typename T>
struct Work {
  T* big = nullptr;               // scratch slabs of the large-cluster kernel
  int64_t big_slab = 0, big_blocks = 0;
  double* xbig = nullptr;         // FP64 slabs of the scaling-and-squaring kernel (De >= 64)
  int64_t xslab = 0, xblocks = 0;
  T* Tb[2] = {nullptr, nullptr};  // partial traces, message layout
  T* Rb[2] = {nullptr, nullptr};  // marginals of clusters with parents
  T* W[4] = {nullptr, nullptr, nullptr, nullptr};  // fused ping-pong state: nu1, ze1, nu2, ze2
  bool fused_ready = false;
};

// A captured chunk fixes every kernel argument at capture time (buffers, launch shapes, Jacobi
// settings, slab counts), so the cache is keyed by the caller's buffers and the problem's settings
// generation, which every settings call advances (dropping the graphs of older generations).
struct GraphKey {
  int prec;
  const void* nu;
  const void* ze;
  uint64_t gen;
  bool operator<(const GraphKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (nu != o.nu) return nu < o.nu;
    if (ze != o.ze) return ze < o.ze;
    return gen < o.gen;
  }
};
constexpr size_t kMaxGraphs = 8;  // captured chunks kept per problem (least recently used evicted)

}  // namespace

// ------------------------------------------------------------------------------------------
// workspace of lrh_certify_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device, with that device
// current, when the first problem is built there, and kept per device.
// ------------------------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::string g_scratch_err[kMaxDevices];

// With `device` current: look up this device's copy of the array (once per device).
void bind_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return;
  }
  g_scratch_ptr[device] = ptr;
}

void* static_scratch(int device, std::string& why) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    why = "device index beyond the static workspace table";
    return nullptr;
  }
  if (!g_scratch_ptr[device]) why = g_scratch_err[device].empty() ? "static workspace not bound" : g_scratch_err[device];
  return g_scratch_ptr[device];
}
}  // namespace

struct lrh_problem_s {
  int device = 0;
  bool host_only = false;  // built with hip_device < 0: poset and layout only
  bool cplx = false;
  int64_t n_clusters = 0, n_msgs = 0, n_inst = 0;
  int max_D = 0;
  // host poset
  std::vector<int64_t> c_ptr;
  std::vector<int32_t> c_sites, c_inst, c_D;
  std::vector<int32_t> m_parent, m_child, m_bucket;
  std::vector<int64_t> m_index;
  std::vector<CBucket> cb;
  std::vector<MBucket> mb;
  double Lambda = 0, Gamma = 0;
  int max_sweeps = 30;
  double tol_override = 0.0;
  int64_t nu_len = 0, R_len = 0, marg_len = 0;
  // device globals
  double* h = nullptr;
  int64_t* inst_ptr = nullptr;
  double* scal = nullptr;
  double* scal2 = nullptr;
  int64_t* marg_off = nullptr;
  unsigned long long* health = nullptr;  // [0] noconv, [1] nonfinite, [2] certificate fallbacks
  int cert_method = 0;                   // lrh_set_certify_method
  int32_t* improved = nullptr;
  double* nu64_tmp = nullptr;            // widened copy of a float nu for certify
  double* cert_ws = nullptr;             // tridiagonals of the 16- and 32-dimensional buckets (certify)
  FusedParams* fp = nullptr;             // [kFusedTableMax]
  // ---- parametrised terms (adjoint) ----
  int64_t n_params = 0;
  double* hfix = nullptr;                // h without the parametrised parts, packed like h
  double* dterm = nullptr;               // packed d h_t / d c blocks
  int64_t n_pc = 0;                      // clusters carrying parametrised terms (CSR)
  int64_t *pc_hoff = nullptr, *pc_ptr = nullptr, *pc_doff = nullptr;
  int32_t *pc_param = nullptr, *pc_ncomp = nullptr;
  int64_t *pp_ptr = nullptr, *pp_yoff = nullptr, *pp_doff = nullptr;  // parameters -> terms (CSR)
  int32_t* pp_D = nullptr;
  int32_t* cinst = nullptr;              // instance of every library cluster
  double* ywork = nullptr;               // per-cluster cotangent Y (marg layout)
  double* ones = nullptr;                // [n_inst] of 1.0
  std::vector<double*> adj_ws;           // reverse-mode workspace
  int64_t adj_T = -1;
  Work<float> w32;
  Work<double> w64;
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, std::pair<hipGraphExec_t, uint64_t>> graphs;  // exec, last use
  uint64_t settings_gen = 0, graph_clock = 0;
  int64_t slab_limit = 0;                // cap on per-workgroup scratch slabs (0: default caps)
  std::vector<void*> allocs;
  std::vector<int32_t> pp_tmp_g;

  ~lrh_problem_s() {
    if (host_only) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second.first);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
    (void)hipSetDevice(cur);
  }

  template <typename T>
  lrh_status dalloc(T** out, int64_t n) {
    *out = nullptr;
    if (n <= 0) return LRH_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)n * sizeof(T));
    if (e != hipSuccess) return fail(LRH_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(p);
    *out = (T*)p;
    return LRH_OK;
  }
  template <typename T>
  lrh_status upload(T** out, const std::vector<T>& v) {
    lrh_status st = dalloc(out, (int64_t)v.size());
    if (st != LRH_OK) return st;
    if (!v.empty()) HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return LRH_OK;
  }
  template <typename T>
  Work<T>& work();
};
template <> Work<float>& lrh_problem_s::work<float>() { return w32; }
template <> Work<double>& lrh_problem_s::work<double>() { return w64; }

namespace {

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

inline int comps_of(int D, bool cplx) { return cplx ? D * D : D * (D + 1) / 2; }

// ------------------------------------------------------------------------------------------
// problem construction
// ------------------------------------------------------------------------------------------

lrh_status build(const lrh_problem_desc* d, lrh_problem_s* P) {
  if (!d) return fail(LRH_E_INVALID, "null problem description");
  const int n = d->n_sites;
  if (n <= 0) return fail(LRH_E_INVALID, "n_sites must be positive");
  if (!d->site_dim) return fail(LRH_E_INVALID, "null site_dim");
  std::vector<int> sd(n);
  for (int i = 0; i < n; ++i) {
    if (d->site_dim[i] != 2 && d->site_dim[i] != 3)
      return fail(LRH_E_UNSUPPORTED, "site dimension must be 2 (spin-1/2) or 3 (spin-1)");
    sd[i] = d->site_dim[i];
  }
  int dmax = 2;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, sd[i]);
  if (d->n_terms < 0 || d->n_top < 0) return fail(LRH_E_INVALID, "negative counts");
  if (d->n_terms > 0 && (!d->term_ptr || !d->term_sites || !d->term_off || !d->term_re))
    return fail(LRH_E_INVALID, "null term arrays");
  if (d->n_top > 0 && (!d->top_ptr || !d->top_sites)) return fail(LRH_E_INVALID, "null top arrays");
  P->cplx = (d->term_im != nullptr);
  std::vector<int32_t> inst(n, 0);
  if (d->site_instance)
    for (int i = 0; i < n; ++i) {
      if (d->site_instance[i] < 0) return fail(LRH_E_INVALID, "negative instance id");
      inst[i] = d->site_instance[i];
    }
  int64_t n_inst = 0;
  for (int i = 0; i < n; ++i) n_inst = std::max<int64_t>(n_inst, inst[i] + 1);
  P->n_inst = n_inst;

  // ---- C_full ----
  std::unordered_map<Key, int32_t, KeyHash> index;
  std::vector<Key> keys;
  auto make_key = [&](const int32_t* s, int k, Key& key) -> lrh_status {
    if (k <= 0) return fail(LRH_E_INVALID, "empty cluster or term support");
    if (k > kMaxSites) return fail(LRH_E_UNSUPPORTED, "cluster with more than 8 sites (D_e > 256)");
    key.k = k;
    int64_t D = 1;
    bool q = true;
    for (int i = 0; i < k; ++i) {
      if (s[i] < 0 || s[i] >= n) return fail(LRH_E_INVALID, "site index out of range");
      if (i > 0 && s[i] <= s[i - 1]) return fail(LRH_E_INVALID, "sites must be ascending and distinct");
      key.s[i] = s[i];
      D *= sd[s[i]];
      q = q && sd[s[i]] == 2;
    }
    if (!q && D > kMaxGenericD) return fail(LRH_E_UNSUPPORTED, "cluster with a spin-1 site and D_e > 64");
    return LRH_OK;
  };
  auto add = [&](const Key& key) {
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    const int32_t id = (int32_t)keys.size();
    index.emplace(key, id);
    keys.push_back(key);
    return id;
  };
  const bool two_level = (d->flags & LRH_TWO_LEVEL) != 0;
  if (two_level && (d->flags & LRH_SUBINTERVALS))
    return fail(LRH_E_INVALID, "LRH_TWO_LEVEL and LRH_SUBINTERVALS exclude each other");
  if (d->flags & ~(LRH_SUBINTERVALS | LRH_TWO_LEVEL)) return fail(LRH_E_INVALID, "unknown problem flag");
  std::vector<int32_t> top_ids;   // C_full id of every distinct top cluster
  for (int c = 0; c < d->n_top; ++c) {
    Key key;
    const int64_t a = d->top_ptr[c], b = d->top_ptr[c + 1];
    lrh_status st = make_key(d->top_sites + a, (int)(b - a), key);
    if (st != LRH_OK) return st;
    const size_t before = keys.size();
    const int32_t id = add(key);
    if (keys.size() > before) top_ids.push_back(id);
    if (d->flags & LRH_SUBINTERVALS) {
      for (int x = 0; x < key.k; ++x)
        for (int y = x + 1; y <= key.k; ++y) {
          Key sub;
          sub.k = y - x;
          for (int i = x; i < y; ++i) sub.s[i - x] = key.s[i];
          add(sub);
        }
    }
  }
  // top clusters holding each site (two-level family)
  std::vector<std::vector<int32_t>> tops_at(two_level ? n : 0);
  if (two_level) {
    for (int32_t id : top_ids)
      for (int i = 0; i < keys[id].k; ++i) tops_at[keys[id].s[i]].push_back(id);
    // maximal pairwise overlaps of top clusters: only tops sharing a site intersect
    std::unordered_map<Key, int32_t, KeyHash> ov_index;
    std::vector<Key> ov;
    for (int v = 0; v < n; ++v) {
      const auto& T = tops_at[v];
      for (size_t x = 0; x < T.size(); ++x)
        for (size_t y = x + 1; y < T.size(); ++y) {
          const Key &A = keys[T[x]], &B = keys[T[y]];
          Key I;
          for (int i = 0, j = 0; i < A.k && j < B.k;) {
            if (A.s[i] == B.s[j]) { I.s[I.k++] = A.s[i]; ++i; ++j; }
            else if (A.s[i] < B.s[j]) ++i;
            else ++j;
          }
          if (I.s[0] != v) continue;   // count each pair once: at its first shared site
          if (ov_index.emplace(I, (int32_t)ov.size()).second) ov.push_back(I);
        }
    }
    // an overlap strictly inside another one shares its first site with it
    std::vector<std::vector<int32_t>> ov_at(n);
    for (size_t o = 0; o < ov.size(); ++o)
      for (int i = 0; i < ov[o].k; ++i) ov_at[ov[o].s[i]].push_back((int32_t)o);
    auto subset = [](const Key& a, const Key& b) {   // a strictly inside b
      if (a.k >= b.k) return false;
      int j = 0;
      for (int i = 0; i < a.k; ++i) {
        while (j < b.k && b.s[j] < a.s[i]) ++j;
        if (j == b.k || b.s[j] != a.s[i]) return false;
      }
      return true;
    };
    for (size_t o = 0; o < ov.size(); ++o) {
      bool maximal = true;
      for (int32_t q : ov_at[ov[o].s[0]])
        if (subset(ov[o], ov[q])) { maximal = false; break; }
      if (maximal) add(ov[o]);
    }
  }
  // homes of every term: the cluster equal to its support, or (two-level family) every
  // top cluster holding the support, each with weight 1 / (number of such tops)
  struct Home { int32_t c; uint8_t pos[8]; double w; };
  std::vector<std::vector<Home>> term_home(d->n_terms);
  for (int t = 0; t < d->n_terms; ++t) {
    Key key;
    const int64_t a = d->term_ptr[t], b = d->term_ptr[t + 1];
    lrh_status st = make_key(d->term_sites + a, (int)(b - a), key);
    if (st != LRH_OK) return st;
    int64_t D = 1;
    for (int i = 0; i < key.k; ++i) D *= sd[key.s[i]];
    if (d->term_off[t + 1] - d->term_off[t] != D * D) return fail(LRH_E_INVALID, "term block size mismatch");
    if (!two_level) {
      Home h{add(key), {0, 1, 2, 3, 4, 5, 6, 7}, 1.0};
      term_home[t].push_back(h);
      continue;
    }
    for (int32_t id : tops_at[key.s[0]]) {
      const Key& T = keys[id];
      Home h{id, {}, 0.0};
      int found = 0;
      for (int i = 0, j = 0; i < key.k && j < T.k; ++j)
        if (T.s[j] == key.s[i]) h.pos[i++] = (uint8_t)j, ++found;
      if (found == key.k) term_home[t].push_back(h);
    }
    if (term_home[t].empty()) return fail(LRH_E_INVALID, "term support lies in no top cluster");
    for (auto& h : term_home[t]) h.w = 1.0 / (double)term_home[t].size();
  }
  if (!two_level)
    for (int v = 0; v < n; ++v) {
      Key key;
      key.k = 1;
      key.s[0] = v;
      add(key);
    }
  const int64_t nc = (int64_t)keys.size();
  if (nc > (int64_t)INT32_MAX / 2) return fail(LRH_E_UNSUPPORTED, "too many clusters");
  // instance of every cluster
  std::vector<int32_t> cinst(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const Key& k = keys[c];
    cinst[c] = inst[k.s[0]];
    for (int i = 1; i < k.k; ++i)
      if (inst[k.s[i]] != cinst[c]) return fail(LRH_E_INVALID, "cluster spans instances");
  }
  // library order: (instance, size, sites)
  std::vector<int32_t> order(nc);
  for (int64_t c = 0; c < nc; ++c) order[c] = (int32_t)c;
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (cinst[a] != cinst[b]) return cinst[a] < cinst[b];
    const Key &ka = keys[a], &kb = keys[b];
    if (ka.k != kb.k) return ka.k < kb.k;
    for (int i = 0; i < ka.k; ++i)
      if (ka.s[i] != kb.s[i]) return ka.s[i] < kb.s[i];
    return false;
  });
  std::vector<int32_t> gid_of(nc);
  for (int64_t g = 0; g < nc; ++g) gid_of[order[g]] = (int32_t)g;
  P->n_clusters = nc;
  P->c_ptr.assign(nc + 1, 0);
  P->c_inst.resize(nc);
  P->c_D.resize(nc);
  for (int64_t g = 0; g < nc; ++g) {
    const Key& k = keys[order[g]];
    P->c_ptr[g + 1] = P->c_ptr[g] + k.k;
    P->c_inst[g] = cinst[order[g]];
    int D = 1;
    for (int i = 0; i < k.k; ++i) D *= sd[k.s[i]];
    P->c_D[g] = D;
    P->max_D = std::max(P->max_D, P->c_D[g]);
  }
  P->c_sites.resize(P->c_ptr[nc]);
  for (int64_t g = 0; g < nc; ++g) {
    const Key& k = keys[order[g]];
    for (int i = 0; i < k.k; ++i) P->c_sites[P->c_ptr[g] + i] = k.s[i];
  }

  // ---- Hasse diagram: maximal proper subsets present in C_full ----
  std::vector<std::vector<std::pair<int32_t, int32_t>>> children(nc);  // (child gid, kernel mask)
  std::vector<std::vector<int32_t>> parents(nc);
  for (int64_t g = 0; g < nc; ++g) {
    const Key& k = keys[order[g]];
    std::vector<std::pair<int32_t, uint32_t>> found;  // (gid, position mask)
    const uint32_t full = (1u << k.k) - 1;
    for (uint32_t pm = 1; pm < full; ++pm) {
      Key sub;
      for (int i = 0; i < k.k; ++i)
        if (pm >> i & 1) sub.s[sub.k++] = k.s[i];
      auto it = index.find(sub);
      if (it != index.end()) found.push_back({gid_of[it->second], pm});
    }
    for (auto& f : found) {
      bool maximal = true;
      for (auto& o : found)
        if (o.second != f.second && (o.second & f.second) == f.second) { maximal = false; break; }
      if (!maximal) continue;
      // position j (0 = first site, most significant) -> kernel bit (k-1-j)
      int32_t kmask = 0;
      for (int j = 0; j < k.k; ++j)
        if (f.second >> j & 1) kmask |= 1 << (k.k - 1 - j);
      children[g].push_back({f.first, kmask});
    }
    std::sort(children[g].begin(), children[g].end());
    for (auto& ch : children[g]) parents[ch.first].push_back((int32_t)g);
  }
  for (auto& p : parents) std::sort(p.begin(), p.end());

  // child dimension per cluster (must be uniform)
  std::vector<int32_t> Dc(nc, 0);
  for (int64_t g = 0; g < nc; ++g) {
    for (auto& ch : children[g]) {
      const int D = P->c_D[ch.first];
      if (Dc[g] == 0) Dc[g] = D;
      else if (Dc[g] != D) return fail(LRH_E_UNSUPPORTED, "cluster whose children have different dimensions");
    }
  }

  // ---- buckets ----
  std::map<std::pair<int, int>, int> cb_index;
  for (int64_t g = 0; g < nc; ++g) cb_index[{P->c_D[g], Dc[g]}] = 0;
  int nb = 0;
  for (auto& kv : cb_index) kv.second = nb++;
  P->cb.resize(nb);
  for (auto& kv : cb_index) {
    P->cb[kv.second].De = kv.first.first;
    P->cb[kv.second].Dc = kv.first.second;
  }
  std::vector<int32_t> cb_of(nc), pos_in_cb(nc);
  for (int64_t g = 0; g < nc; ++g) {
    const int b = cb_index[{P->c_D[g], Dc[g]}];
    cb_of[g] = b;
    pos_in_cb[g] = (int32_t)P->cb[b].h_gid.size();
    P->cb[b].h_gid.push_back((int32_t)g);
  }
  for (auto& B : P->cb) {
    int shapes[8];
    if (cluster_shapes(B.De, B.Dc, false, P->cplx, MODE_GIBBS, shapes) > 0) B.W = shapes[0];
    if (cluster_shapes(B.De, B.Dc, true, P->cplx, MODE_GIBBS, shapes) > 0) B.W64 = shapes[0];
    B.n = (int64_t)B.h_gid.size();
    for (int32_t g : B.h_gid) {
      B.maxch = std::max<int>(B.maxch, (int)children[g].size());
      B.maxpar = std::max<int>(B.maxpar, (int)parents[g].size());
    }
  }
  // message buckets by child dimension
  std::map<int, int> mb_index;
  for (int64_t g = 0; g < nc; ++g)
    for (auto& ch : children[g]) mb_index[P->c_D[ch.first]] = 0;
  int nmb = 0;
  for (auto& kv : mb_index) kv.second = nmb++;
  if (nmb > LRH_MAX_BUCKETS) return fail(LRH_E_UNSUPPORTED, "too many message buckets");
  P->mb.resize(nmb);
  for (auto& kv : mb_index) {
    P->mb[kv.second].D = kv.first;
    P->mb[kv.second].comps = comps_of(kv.first, P->cplx);
  }
  for (auto& B : P->cb) {
    if (B.Dc > 0) B.mb_child = mb_index[B.Dc];
    auto it = mb_index.find(B.De);
    if (it != mb_index.end()) B.mb_self = it->second;
  }
  // message numbering: per child bucket, slot-major over each parent cluster bucket so
  // lanes of consecutive parents read consecutive messages
  std::vector<std::vector<int32_t>> h_ch(nb), h_chmask(nb), h_par(nb);
  for (int b = 0; b < nb; ++b) {
    h_ch[b].assign((size_t)P->cb[b].maxch * P->cb[b].n, -1);
    h_chmask[b].assign((size_t)P->cb[b].maxch * P->cb[b].n, 0);
    h_par[b].assign((size_t)P->cb[b].maxpar * P->cb[b].n, -1);
  }
  std::map<std::pair<int32_t, int32_t>, int64_t> msg_of;  // (parent gid, child gid) -> index in bucket
  for (int mbi = 0; mbi < nmb; ++mbi) {
    MBucket& M = P->mb[mbi];
    int64_t cnt = 0;
    for (int b = 0; b < nb; ++b) {
      CBucket& B = P->cb[b];
      if (B.mb_child != mbi) continue;
      for (int s = 0; s < B.maxch; ++s)
        for (int64_t c = 0; c < B.n; ++c) {
          const int32_t g = B.h_gid[c];
          if ((int)children[g].size() <= s) continue;
          const int64_t idx = cnt++;
          if (idx > INT32_MAX) return fail(LRH_E_UNSUPPORTED, "too many messages in a bucket");
          h_ch[b][(size_t)s * B.n + c] = (int32_t)idx;
          h_chmask[b][(size_t)s * B.n + c] = children[g][s].second;
          msg_of[{g, children[g][s].first}] = idx;
          P->m_parent.push_back(g);
          P->m_child.push_back(children[g][s].first);
          P->m_bucket.push_back(mbi);
          P->m_index.push_back(idx);
        }
    }
    M.M = cnt;
  }
  // reorder the exported message list into (bucket, index) order
  {
    std::vector<size_t> perm(P->m_parent.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
    std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
      if (P->m_bucket[a] != P->m_bucket[b]) return P->m_bucket[a] < P->m_bucket[b];
      return P->m_index[a] < P->m_index[b];
    });
    auto apply = [&](auto& v) {
      auto w = v;
      for (size_t i = 0; i < perm.size(); ++i) w[i] = v[perm[i]];
      v.swap(w);
    };
    apply(P->m_parent);
    apply(P->m_child);
    apply(P->m_bucket);
    apply(P->m_index);
  }
  P->n_msgs = (int64_t)P->m_parent.size();
  int64_t off = 0;
  for (auto& M : P->mb) {
    M.offset = off;
    off += M.M * M.comps;
  }
  P->nu_len = off;
  // parent messages per cluster
  for (int b = 0; b < nb; ++b) {
    CBucket& B = P->cb[b];
    for (int64_t c = 0; c < B.n; ++c) {
      const int32_t g = B.h_gid[c];
      for (size_t s = 0; s < parents[g].size(); ++s)
        h_par[b][s * B.n + c] = (int32_t)msg_of[{parents[g][s], g}];
    }
  }
  // marginal slots: clusters with parents, per dimension
  std::vector<int32_t> rslot(nc, -1);
  for (int mbi = 0; mbi < nmb; ++mbi) {
    MBucket& M = P->mb[mbi];
    int64_t S = 0;
    for (int64_t g = 0; g < nc; ++g)
      if (P->c_D[g] == M.D && !parents[g].empty()) rslot[g] = (int32_t)S++;
    M.S = S;
    M.comps_r = comps_of(M.D, P->cplx);
  }
  int64_t roff = 0;
  for (auto& M : P->mb) {
    M.roff = roff;
    roff += M.S * M.comps_r;
  }
  P->R_len = roff;

  // ---- h_e: the terms at home in the cluster, lifted and weighted, packed ----
  // H += w * (1 (x) B): B (Dt x Dt) acts on the cluster's sites at positions pos[0..kt); a cluster
  // index is the big-endian mixed-radix number of its sites' states (first site most significant)
  auto lift_add = [&](std::vector<std::complex<double>>& H, const Key& ck, const Home& h, int kt, const double* re,
                      const double* im, double scale) {
    const int ke = ck.k;
    int de[8], stride[8], tst[8];
    int De = 1;
    for (int p = ke - 1; p >= 0; --p) {
      de[p] = sd[ck.s[p]];
      stride[p] = De;
      De *= de[p];
    }
    int Dt = 1;
    for (int j = kt - 1; j >= 0; --j) {
      tst[j] = Dt;
      Dt *= de[h.pos[j]];
    }
    for (int i = 0; i < De; ++i) {
      int a = 0, base = i;
      for (int j = 0; j < kt; ++j) {
        const int dg = (i / stride[h.pos[j]]) % de[h.pos[j]];
        a += dg * tst[j];
        base -= dg * stride[h.pos[j]];
      }
      for (int b = 0; b < Dt; ++b) {
        int jj = base;
        for (int j = 0; j < kt; ++j) jj += ((b / tst[j]) % de[h.pos[j]]) * stride[h.pos[j]];
        H[(size_t)i * De + jj] += scale * h.w * std::complex<double>(re[a * Dt + b], im ? im[a * Dt + b] : 0.0);
      }
    }
  };
  std::vector<std::vector<std::complex<double>>> hdense(nc);
  for (int t = 0; t < d->n_terms; ++t) {
    const int kt = (int)(d->term_ptr[t + 1] - d->term_ptr[t]);
    int D = 1;
    for (int64_t q = d->term_ptr[t]; q < d->term_ptr[t + 1]; ++q) D *= sd[d->term_sites[q]];
    const double* re = d->term_re + d->term_off[t];
    const double* im = d->term_im ? d->term_im + d->term_off[t] : nullptr;
    double mx = 0;
    for (int i = 0; i < D * D; ++i) mx = std::max(mx, std::abs(std::complex<double>(re[i], im ? im[i] : 0)));
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        std::complex<double> a(re[i * D + j], im ? im[i * D + j] : 0.0);
        std::complex<double> b(re[j * D + i], im ? -im[j * D + i] : 0.0);
        if (std::abs(a - b) > 1e-12 * std::max(1.0, mx)) return fail(LRH_E_INVALID, "term is not Hermitian");
      }
    for (const Home& h : term_home[t]) {
      const int32_t g = gid_of[h.c];
      const int De = P->c_D[g];
      auto& H = hdense[g];
      if (H.empty()) H.assign((size_t)De * De, 0.0);
      lift_add(H, keys[h.c], h, kt, re, im, 1.0);
    }
  }
  std::vector<double> hpack;
  std::vector<std::vector<int64_t>> h_hoff(nb);
  for (int b = 0; b < nb; ++b) h_hoff[b].assign(P->cb[b].n, -1);
  for (int64_t g = 0; g < nc; ++g) {
    if (hdense[g].empty()) continue;
    const int D = P->c_D[g];
    h_hoff[cb_of[g]][pos_in_cb[g]] = (int64_t)hpack.size();
    const auto& H = hdense[g];
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j) hpack.push_back(0.5 * (H[i * D + j].real() + H[j * D + i].real()));
    if (P->cplx)
      for (int i = 0; i < D; ++i)
        for (int j = i + 1; j < D; ++j) hpack.push_back(0.5 * (H[i * D + j].imag() - H[j * D + i].imag()));
  }

  // ---- parametrised terms ----
  std::vector<double> hfix_pack, dterm_pack;
  std::vector<int64_t> pc_hoff, pc_ptr, pc_doff, pp_ptr, pp_yoff, pp_doff;
  std::vector<int32_t> pc_param, pc_ncomp, pp_D;
  if (d->n_params < 0) return fail(LRH_E_INVALID, "negative n_params");
  P->n_params = d->n_params;
  if (d->n_params > 0) {
    if (!d->term_param || !d->dterm_re || !d->params) return fail(LRH_E_INVALID, "null parameter arrays");
    if (P->cplx != (d->dterm_im != nullptr)) return fail(LRH_E_INVALID, "dterm_im must match term_im");
    hfix_pack = hpack;
    struct PT { int32_t g; int32_t p; int32_t t; int64_t doff; };
    std::vector<PT> pts;
    for (int t = 0; t < d->n_terms; ++t) {
      const int32_t pidx = d->term_param[t];
      if (pidx < 0) continue;
      if (pidx >= d->n_params) return fail(LRH_E_INVALID, "term_param out of range");
      const int kt = (int)(d->term_ptr[t + 1] - d->term_ptr[t]);
      int Dt = 1;
      for (int64_t q = d->term_ptr[t]; q < d->term_ptr[t + 1]; ++q) Dt *= sd[d->term_sites[q]];
      const double* re = d->dterm_re + d->term_off[t];
      const double* im = d->dterm_im ? d->dterm_im + d->term_off[t] : nullptr;
      for (int i = 0; i < Dt; ++i)
        for (int j = 0; j < Dt; ++j) {
          std::complex<double> a(re[i * Dt + j], im ? im[i * Dt + j] : 0.0);
          std::complex<double> b(re[j * Dt + i], im ? -im[j * Dt + i] : 0.0);
          if (std::abs(a - b) > 1e-12 * std::max(1.0, std::abs(a))) return fail(LRH_E_INVALID, "dterm is not Hermitian");
        }
      for (const Home& h : term_home[t]) {
        const int32_t g = gid_of[h.c];
        const int D = P->c_D[g];
        std::vector<std::complex<double>> B((size_t)D * D, 0.0);
        lift_add(B, keys[h.c], h, kt, re, im, 1.0);
        const int64_t doff = (int64_t)dterm_pack.size();
        for (int i = 0; i < D; ++i)
          for (int j = i; j < D; ++j) dterm_pack.push_back(0.5 * (B[i * D + j].real() + B[j * D + i].real()));
        if (P->cplx)
          for (int i = 0; i < D; ++i)
            for (int j = i + 1; j < D; ++j) dterm_pack.push_back(0.5 * (B[i * D + j].imag() - B[j * D + i].imag()));
        // constant part of the cluster: subtract params[p] * dterm
        const int64_t ho = h_hoff[cb_of[g]][pos_in_cb[g]];
        const int nco = comps_of(D, P->cplx);
        for (int k = 0; k < nco; ++k) hfix_pack[ho + k] -= d->params[pidx] * dterm_pack[doff + k];
        pts.push_back({g, pidx, t, doff});
      }
    }
    // clusters -> terms
    std::vector<PT> byc = pts;
    std::stable_sort(byc.begin(), byc.end(), [](const PT& a, const PT& b) { return a.g < b.g; });
    for (size_t i = 0; i < byc.size(); ++i) {
      if (i == 0 || byc[i].g != byc[i - 1].g) {
        pc_ptr.push_back((int64_t)i);
        const int32_t g = byc[i].g;
        pc_hoff.push_back(h_hoff[cb_of[g]][pos_in_cb[g]]);
        pc_ncomp.push_back(comps_of(P->c_D[g], P->cplx));
      }
      pc_param.push_back(byc[i].p);
      pc_doff.push_back(byc[i].doff);
    }
    pc_ptr.push_back((int64_t)byc.size());
    P->n_pc = (int64_t)pc_hoff.size();
    // parameters -> terms
    std::vector<PT> byp = pts;
    std::stable_sort(byp.begin(), byp.end(), [](const PT& a, const PT& b) { return a.p < b.p; });
    pp_ptr.assign(d->n_params + 1, 0);
    for (auto& x : byp) pp_ptr[x.p + 1]++;
    for (int q = 0; q < d->n_params; ++q) pp_ptr[q + 1] += pp_ptr[q];
    for (auto& x : byp) {
      pp_doff.push_back(x.doff);
      pp_D.push_back(P->c_D[x.g]);
      pp_yoff.push_back(-1);  // filled below once marginal offsets are known
    }
    // remember the cluster of each entry for the Y offset
    std::vector<int32_t> pp_g;
    for (auto& x : byp) pp_g.push_back(x.g);
    P->pp_tmp_g.swap(pp_g);
  }

  // ---- per-instance cluster ranges, marginal offsets ----
  std::vector<int64_t> inst_ptr(n_inst + 1, 0);
  for (int64_t g = 0; g < nc; ++g) inst_ptr[P->c_inst[g] + 1]++;
  for (int64_t i = 0; i < n_inst; ++i) inst_ptr[i + 1] += inst_ptr[i];
  std::vector<int64_t> marg_off(nc);
  int64_t moff = 0;
  for (int64_t g = 0; g < nc; ++g) {
    marg_off[g] = moff;
    moff += comps_of(P->c_D[g], P->cplx);
  }
  P->marg_len = moff;
  for (size_t i = 0; i < pp_yoff.size(); ++i) pp_yoff[i] = marg_off[P->pp_tmp_g[i]];

  // ---- Lipschitz factor Lambda_G and Gamma_G ----
  bool two_local = true;
  for (int64_t g = 0; g < nc; ++g)
    if (P->c_ptr[g + 1] - P->c_ptr[g] > 2) two_local = false;
  if (two_local) {
    size_t deg = 0;
    for (int64_t g = 0; g < nc; ++g)
      if (P->c_ptr[g + 1] - P->c_ptr[g] == 1) deg = std::max(deg, parents[g].size());
    P->Lambda = (double)deg + (double)dmax;  // Delta_G + d
  } else {
    double lam = 0;
    for (size_t m = 0; m < P->m_parent.size(); ++m) {
      const int32_t e = P->m_parent[m], f = P->m_child[m];
      const double me = (double)(parents[e].size() + children[e].size());
      const double mf = (double)(parents[f].size() + children[f].size());
      lam = std::max(lam, mf + me * P->c_D[e] / (double)P->c_D[f]);
    }
    P->Lambda = lam;
  }
  double gam = 0;
  for (int64_t g = 0; g < nc; ++g) gam += std::log((double)P->c_D[g]);
  P->Gamma = gam;

  if (P->host_only) return LRH_OK;
  // ---- device upload ----
  lrh_status st;
#define UP(dst, vec)                      \
  do {                                    \
    st = P->upload(&(dst), vec);          \
    if (st != LRH_OK) return st;          \
  } while (0)
  // marginal slot of every message's child, per message bucket
  std::vector<std::vector<int32_t>> h_mrs(nmb);
  {
    size_t pos = 0;
    for (int mbi = 0; mbi < nmb; ++mbi) {
      h_mrs[mbi].resize(P->mb[mbi].M);
      for (int64_t m = 0; m < P->mb[mbi].M; ++m, ++pos) h_mrs[mbi][m] = rslot[P->m_child[pos]];
    }
  }
  for (int b = 0; b < nb; ++b) {
    CBucket& B = P->cb[b];
    std::vector<int32_t> rs(B.n);
    for (int64_t c = 0; c < B.n; ++c) rs[c] = rslot[B.h_gid[c]];
    std::vector<int32_t> chrs(h_ch[b].size(), -1);
    if (B.mb_child >= 0)
      for (size_t i = 0; i < chrs.size(); ++i)
        if (h_ch[b][i] >= 0) chrs[i] = h_mrs[B.mb_child][h_ch[b][i]];
    if (chrs.empty()) chrs.push_back(-1);
    UP(B.chrs, chrs);
    if (generic_dim(B.De) && B.maxch > 0) {
      // per (child slot, cluster, cluster index i): i's child index a and remaining index r, and the
      // cluster index of the child/remainder pair (a, r) = (i / NR, i % NR), NR = De / Dc
      std::vector<int32_t> gt((size_t)B.maxch * B.n * B.De, 0);
      for (int sl = 0; sl < B.maxch; ++sl)
        for (int64_t c = 0; c < B.n; ++c) {
          if (h_ch[b][(size_t)sl * B.n + c] < 0) continue;
          const int32_t g = B.h_gid[c];
          const int k = (int)(P->c_ptr[g + 1] - P->c_ptr[g]);
          const int32_t kmask = h_chmask[b][(size_t)sl * B.n + c];
          int de[8], stride[8];
          int De = 1;
          for (int p = k - 1; p >= 0; --p) {
            de[p] = sd[P->c_sites[P->c_ptr[g] + p]];
            stride[p] = De;
            De *= de[p];
          }
          int Dc = 1;
          for (int p = 0; p < k; ++p)
            if (kmask >> (k - 1 - p) & 1) Dc *= de[p];
          const int NR = De / Dc;
          int32_t* out = gt.data() + ((size_t)sl * B.n + c) * B.De;
          for (int i = 0; i < De; ++i) {
            int a = 0, r = 0;
            for (int p = 0; p < k; ++p) {
              const int dg = (i / stride[p]) % de[p];
              if (kmask >> (k - 1 - p) & 1) a = a * de[p] + dg;
              else r = r * de[p] + dg;
            }
            out[i] |= a | (r << 8);
            out[a * NR + r] |= i << 16;
          }
        }
      UP(B.gtab, gt);
    }
    UP(B.gid, B.h_gid);
    UP(B.hoff, h_hoff[b]);
    UP(B.ch, h_ch[b]);
    UP(B.chmask, h_chmask[b]);
    UP(B.par, h_par[b]);
    UP(B.rslot, rs);
  }
  {
    size_t pos = 0;
    for (int mbi = 0; mbi < nmb; ++mbi) {
      MBucket& M = P->mb[mbi];
      std::vector<int32_t> rs(M.M), mi(M.M);
      for (int64_t m = 0; m < M.M; ++m, ++pos) {
        rs[m] = rslot[P->m_child[pos]];
        mi[m] = P->c_inst[P->m_parent[pos]];
      }
      UP(M.rslot, rs);
      UP(M.inst, mi);
    }
  }
  if (hpack.empty()) hpack.push_back(0.0);
  UP(P->h, hpack);
  UP(P->inst_ptr, inst_ptr);
  UP(P->cinst, P->c_inst);
  if (P->n_params > 0) {
    UP(P->hfix, hfix_pack);
    UP(P->dterm, dterm_pack);
    UP(P->pc_hoff, pc_hoff);
    UP(P->pc_ptr, pc_ptr);
    UP(P->pc_param, pc_param);
    UP(P->pc_doff, pc_doff);
    UP(P->pc_ncomp, pc_ncomp);
    UP(P->pp_ptr, pp_ptr);
    UP(P->pp_yoff, pp_yoff);
    UP(P->pp_doff, pp_doff);
    UP(P->pp_D, pp_D);
  }
  UP(P->marg_off, marg_off);
  st = P->dalloc(&P->scal, nc);
  if (st != LRH_OK) return st;
  st = P->dalloc(&P->scal2, nc);
  if (st != LRH_OK) return st;
  st = P->dalloc(&P->health, 3);
  if (st != LRH_OK) return st;
  HIP_TRY(hipMemset(P->health, 0, 3 * sizeof(unsigned long long)));
  st = P->dalloc(&P->improved, std::max<int64_t>(n_inst, 1));
  if (st != LRH_OK) return st;
  st = P->dalloc(&P->fp, kFusedTableMax);
  if (st != LRH_OK) return st;
#undef UP
  return LRH_OK;
}

// ------------------------------------------------------------------------------------------
// drivers
// ------------------------------------------------------------------------------------------

template <typename T>
lrh_status ensure_work(lrh_problem_s* P, bool fused) {
  Work<T>& w = P->work<T>();
  lrh_status st;
  if (P->slab_limit > 0) {   // slabs allocated before a limit was set: use only the first ones
    w.big_blocks = std::min<int64_t>(w.big_blocks, P->slab_limit);
    w.xblocks = std::min<int64_t>(w.xblocks, P->slab_limit);
  }
  if (!w.big) {
    int64_t nbig = 0;
    int Dmax = 0;
    for (const CBucket& B : P->cb)
      if (B.De >= 128) {
        nbig = std::max<int64_t>(nbig, B.n);
        Dmax = std::max(Dmax, B.De);
      }
    if (nbig > 0) {
      w.big_slab = (int64_t)(P->cplx ? 6 : 3) * Dmax * Dmax;
      w.big_blocks = std::min<int64_t>(nbig, P->slab_limit > 0 ? std::min<int64_t>(P->slab_limit, 512) : 512);
      if ((st = P->dalloc(&w.big, w.big_slab * w.big_blocks)) != LRH_OK) return st;
    }
  }
  if (!w.xbig) {
    int64_t nx = 0;
    int Dmax = 0;
    for (const CBucket& B : P->cb)
      if (B.De >= 32) {
        nx = std::max<int64_t>(nx, B.n);
        Dmax = std::max(Dmax, B.De);
      }
    if (nx > 0) {
      w.xslab = (int64_t)5 * (P->cplx ? 2 : 1) * Dmax * Dmax;
      const int64_t cap = Dmax >= 256 ? 512 : 1024;
      w.xblocks = std::min<int64_t>(nx, P->slab_limit > 0 ? std::min<int64_t>(P->slab_limit, cap) : cap);
      if ((st = P->dalloc(&w.xbig, w.xslab * w.xblocks)) != LRH_OK) return st;
    }
  }
  if (!w.Tb[0]) {
    if ((st = P->dalloc(&w.Tb[0], std::max<int64_t>(P->nu_len, 1))) != LRH_OK) return st;
    if ((st = P->dalloc(&w.Rb[0], std::max<int64_t>(P->R_len, 1))) != LRH_OK) return st;
  }
  if (fused && !w.fused_ready) {
    if ((st = P->dalloc(&w.Tb[1], std::max<int64_t>(P->nu_len, 1))) != LRH_OK) return st;
    if ((st = P->dalloc(&w.Rb[1], std::max<int64_t>(P->R_len, 1))) != LRH_OK) return st;
    for (int i = 0; i < 4; ++i)
      if ((st = P->dalloc(&w.W[i], std::max<int64_t>(P->nu_len, 1))) != LRH_OK) return st;
    w.fused_ready = true;
  }
  return LRH_OK;
}

// Doubles of the certification workspace: the tridiagonal (d, |e|^2) of every cluster of the largest
// 16- or 32-dimensional bucket (buckets are certified one after another).
int64_t cert_ws_len(const lrh_problem_s* P) {
  int64_t len = 0;
  for (const CBucket& B : P->cb)
    if (B.De == 16 || B.De == 32) len = std::max<int64_t>(len, (int64_t)2 * B.De * B.n);
  return len;
}

template <typename T>
double default_tol();
template <> double default_tol<float>() { return 4.0 * 1.1920928955078125e-07; }
template <> double default_tol<double>() { return 4.0 * 2.220446049250313e-16; }

// The bucket's chosen shape if it is compiled for this precision / mode, else the first that is.
int shape_for(const lrh_problem_s* P, const CBucket& B, bool dbl, int mode) {
  int shapes[8];
  const int n = cluster_shapes(B.De, B.Dc, dbl, P->cplx, mode, shapes);
  if (mode == MODE_CERTIFY)
    for (int i = 0; i < n; ++i)
      if (shapes[i] == 2) return 2;   // eigenvalues only: tridiagonalisation whenever compiled
  const int want = dbl ? B.W64 : B.W;
  for (int i = 0; i < n; ++i)
    if (shapes[i] == want) return want;
  return n > 0 ? shapes[0] : 64;
}

template <typename T>
ClusterArgs<T> base_args(lrh_problem_s* P, const CBucket& B) {
  ClusterArgs<T> a{};
  a.n = B.n;
  a.De = B.De;
  a.Dc = B.Dc;
  a.maxch = B.maxch;
  a.maxpar = B.maxpar;
  a.gid = B.gid;
  a.hoff = B.hoff;
  a.ch = B.ch;
  a.chmask = B.chmask;
  a.ch_rslot = B.chrs;
  a.gtab = B.gtab;
  a.par = B.par;
  a.rslot = B.rslot;
  a.h = P->h;
  a.scal = P->scal;
  a.scal2 = P->scal2;
  a.tau_rel = 1e-9;
  a.max_sweeps = P->max_sweeps;
  a.tol = P->tol_override > 0 ? P->tol_override : default_tol<T>();
  a.noconv = P->health;
  a.nonfinite = P->health + 1;
  a.cert_fallback = P->health + 2;
  a.cert_method = P->cert_method;
  if (B.mb_child >= 0) a.Mc = P->mb[B.mb_child].M;
  if (B.mb_self >= 0) {
    a.Mp = P->mb[B.mb_self].M;
    a.S = P->mb[B.mb_self].S;
  }
  if (B.De >= 128) {
    Work<T>& w = P->work<T>();
    a.big_scratch = w.big;
    a.big_slab = w.big_slab;
    a.big_blocks = w.big_blocks;
  }
  if (B.De >= 32) {
    Work<T>& w = P->work<T>();
    a.expm_scratch = w.xbig;
    a.expm_slab = w.xslab;
    a.expm_blocks = w.xblocks;
  }
  return a;
}

// One plain pass of the cluster kernels over every bucket at (nu, zeta, theta).
template <typename T>
ClusterArgs<T> pass_args(lrh_problem_s* P, const CBucket& B, const T* nu, const T* ze, double theta, double beta,
                         T* marg, const FusedParams* tab) {
  Work<T>& w = P->work<T>();
  ClusterArgs<T> a = base_args<T>(P, B);
  if (B.mb_child >= 0) {
    const MBucket& M = P->mb[B.mb_child];
    a.nu_c = nu + M.offset;
    a.ze_c = ze ? ze + M.offset : nullptr;
    a.Tout = w.Tb[0] + M.offset;
  }
  if (B.mb_self >= 0) {
    const MBucket& M = P->mb[B.mb_self];
    a.nu_p = nu + M.offset;
    a.ze_p = ze ? ze + M.offset : nullptr;
    a.R = w.Rb[0] + M.roff;
  }
  a.marg = marg;
  a.marg_off = P->marg_off;
  a.beta = beta;
  a.theta = theta;
  a.tab = tab;
  return a;
}

template <typename T>
lrh_status cluster_pass(lrh_problem_s* P, const T* nu, const T* ze, double theta, int mode, double beta,
                        T* marg, hipStream_t s, const FusedParams* tab = nullptr) {
  for (const CBucket& B : P->cb) {
    ClusterArgs<T> a = pass_args<T>(P, B, nu, ze, theta, beta, marg, tab);
    HIP_TRY(launch_cluster<T>(a, P->cplx, mode, B.block, shape_for(P, B, sizeof(T) == 8, mode), s));
  }
  return LRH_OK;
}

// Average duration of one cluster-kernel launch per bucket at messages nu (eta = nu), in the
// bucket's current shape, timed with events on the caller's stream.
template <typename T>
lrh_status time_buckets_t(lrh_problem_s* P, const T* nu, double beta, int reps, double* us, hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  const int mode = beta > 0 ? MODE_GIBBS : MODE_GROUND;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (size_t b = 0; b < P->cb.size(); ++b) {
    const CBucket& B = P->cb[b];
    ClusterArgs<T> a = pass_args<T>(P, B, nu, nullptr, 0.0, beta, nullptr, nullptr);
    const int W = shape_for(P, B, sizeof(T) == 8, mode);
    HIP_TRY(launch_cluster<T>(a, P->cplx, mode, B.block, W, s));
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIP_TRY(launch_cluster<T>(a, P->cplx, mode, B.block, W, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    us[b] = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return LRH_OK;
}

template <typename T>
MsgArgs<T> msg_args(lrh_problem_s* P, const MBucket& M) {
  Work<T>& w = P->work<T>();
  MsgArgs<T> a{};
  a.M = M.M;
  a.comps = M.comps;
  a.S = M.S;
  a.rslot = M.rslot;
  a.inst = M.inst;
  a.R = w.Rb[0] + M.roff;
  a.Tm = w.Tb[0] + M.offset;
  return a;
}

template <typename T>
lrh_status time_messages_t(lrh_problem_s* P, T* nu, T* ze, double beta, int reps, double* us, hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  // one Gibbs pass at the given messages fills the partial traces and marginals the update reads
  if ((st = cluster_pass<T>(P, nu, nullptr, 0.0, MODE_GIBBS, beta, nullptr, s)) != LRH_OK) return st;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (size_t b = 0; b < P->mb.size(); ++b) {
    const MBucket& M = P->mb[b];
    MsgArgs<T> a = msg_args<T>(P, M);
    a.nu = nu + M.offset;
    a.ze = ze + M.offset;
    a.theta = 1.0;
    a.inv_thL = 1e-3;
    HIP_TRY(launch_msg<T>(a, MSG_NESTEROV, 256, s));
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIP_TRY(launch_msg<T>(a, MSG_NESTEROV, 256, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    us[b] = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return LRH_OK;
}

template <typename T>
lrh_status dual_eval_t(lrh_problem_s* P, const T* nu, double beta, double* q, T* grad, T* marg,
                       hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  const int mode = beta > 0 ? MODE_GIBBS : MODE_GROUND;
  if ((st = cluster_pass<T>(P, nu, nullptr, 0.0, mode, beta, marg, s)) != LRH_OK) return st;
  HIP_TRY(launch_reduce(P->scal, P->inst_ptr, P->n_inst, q, nullptr, nullptr, nullptr, nullptr, nullptr, s));
  if (grad) {
    for (const MBucket& M : P->mb) {
      MsgArgs<T> a = msg_args<T>(P, M);
      a.grad = grad + M.offset;
      HIP_TRY(launch_msg<T>(a, MSG_GRAD, 256, s));
    }
  }
  return LRH_OK;
}

template <typename T>
lrh_status subgrad_t(lrh_problem_s* P, T* nu, T* nu_best, double* q_best, int64_t k0, int n_iter, int kind,
                     double scale, double* q_hist, hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  for (int j = 0; j < n_iter; ++j) {
    const int64_t k = k0 + j;
    const double alpha = kind == 0 ? scale / std::sqrt((double)k + 1.0) : scale;
    if ((st = cluster_pass<T>(P, nu, nullptr, 0.0, MODE_GROUND, 0.0, nullptr, s)) != LRH_OK) return st;
    HIP_TRY(launch_reduce(P->scal, P->inst_ptr, P->n_inst, nullptr, nullptr, nullptr, q_best, P->improved,
                          q_hist ? q_hist + (int64_t)j * P->n_inst : nullptr, s));
    for (const MBucket& M : P->mb) {
      MsgArgs<T> a = msg_args<T>(P, M);
      a.nu = nu + M.offset;
      a.nu_best = nu_best + M.offset;
      a.improved = P->improved;
      a.alpha = alpha;
      HIP_TRY(launch_msg<T>(a, MSG_SUBGRAD, 256, s));
    }
  }
  return LRH_OK;
}

double theta_next(double th) { return (std::sqrt(th * th * th * th + 4.0 * th * th) - th * th) / 2.0; }

template <typename T>
lrh_status nesterov_plain(lrh_problem_s* P, T* nu, T* ze, lrh_nesterov_state* stt, int n_iter,
                          hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  for (int j = 0; j < n_iter; ++j) {
    const double th = stt->theta;
    if ((st = cluster_pass<T>(P, nu, ze, th, MODE_GIBBS, stt->beta, nullptr, s)) != LRH_OK) return st;
    for (const MBucket& M : P->mb) {
      MsgArgs<T> a = msg_args<T>(P, M);
      a.nu = nu + M.offset;
      a.ze = ze + M.offset;
      a.theta = th;
      a.inv_thL = 1.0 / (th * stt->L);
      HIP_TRY(launch_msg<T>(a, MSG_NESTEROV, 256, s));
    }
    stt->theta = theta_next(th);
    stt->k += 1;
  }
  return LRH_OK;
}

// Destroy every captured chunk (after the device has finished with them).
void drop_graphs(lrh_problem_s* P) {
  if (P->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& g : P->graphs) (void)hipGraphExecDestroy(g.second.first);
  P->graphs.clear();
}

// Settings that captured chunks bake into their kernel arguments changed: start a new generation.
void settings_changed(lrh_problem_s* P) {
  ++P->settings_gen;
  if (!P->host_only) {
    DeviceGuard guard(P->device);
    drop_graphs(P);
  }
}

// Launch the captured chunk for `key`, capturing it first (enqueue(stream) records the chunk's
// launches).  At most kMaxGraphs chunks are kept; the least recently used one is evicted.
template <typename F>
lrh_status launch_cached_graph(lrh_problem_s* P, const GraphKey& key, hipStream_t s, F&& enqueue) {
  auto it = P->graphs.find(key);
  if (it == P->graphs.end()) {
    if (P->graphs.size() >= kMaxGraphs) {
      auto lru = P->graphs.begin();
      for (auto jt = P->graphs.begin(); jt != P->graphs.end(); ++jt)
        if (jt->second.second < lru->second.second) lru = jt;
      HIP_TRY(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(lru->second.first);
      P->graphs.erase(lru);
    }
    if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed));
    lrh_status est = enqueue(P->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(P->cap_stream, &graph);
    if (est != LRH_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return est;
    }
    if (ee != hipSuccess) return fail(LRH_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(LRH_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    it = P->graphs.emplace(key, std::make_pair(exec, uint64_t(0))).first;
  }
  it->second.second = ++P->graph_clock;
  HIP_TRY(hipGraphLaunch(it->second.first, s));
  return LRH_OK;
}

bool fusable(const lrh_problem_s* P) {
  if (P->mb.size() != 1 || P->mb[0].D != 2) return false;
  for (const CBucket& B : P->cb)
    if (!((B.De == 4 && B.Dc == 2) || (B.De == 2 && B.Dc == 0))) return false;
  return true;
}

// Enqueue one fused segment of n iterations (kernels read their scalars from P->fp[j]).
// Kernel j: state S_j-1 -> S_j (S_0 = user buffers, S_j = W[(j-1)%2] for j >= 1), writes
// T/R of iteration j into buffer j%2; a final message kernel moves S_{n-1} + g into the
// user buffers.
template <typename T>
lrh_status fused_enqueue(lrh_problem_s* P, T* nu, T* ze, int n, hipStream_t s) {
  Work<T>& w = P->work<T>();
  const CBucket* E = nullptr;
  const CBucket* Sb = nullptr;
  for (const CBucket& B : P->cb) {
    if (B.De == 4) E = &B;
    else Sb = &B;
  }
  const MBucket& M = P->mb[0];
  auto state = [&](int j, int which) -> T* {  // which: 0 nu, 1 ze
    if (j == 0) return which == 0 ? nu : ze;
    return w.W[((j - 1) % 2) * 2 + which];
  };
  for (int j = 0; j < n; ++j) {
    const int cur = j % 2, prv = (j + 1) % 2;
    ClusterArgs<T> ea{}, sa{};
    if (E) ea = base_args<T>(P, *E);
    if (Sb) sa = base_args<T>(P, *Sb);
    for (ClusterArgs<T>* a : {&ea, &sa}) {
      a->fp = P->fp + j;
      a->fused_first = (j == 0) ? 1 : 0;
      a->nu_c_prev = state(j == 0 ? 0 : j - 1, 0);
      a->ze_c_prev = state(j == 0 ? 0 : j - 1, 1);
      a->nu_p_prev = a->nu_c_prev;
      a->ze_p_prev = a->ze_c_prev;
      a->Tprev_c = w.Tb[prv];
      a->Rprev_c = w.Rb[prv];
      a->Tprev_p = w.Tb[prv];
      a->Rprev_p = w.Rb[prv];
      a->rslot_of_msg_c = M.rslot;
      a->Sc = M.S;
      a->nu_c_new = (j == 0) ? nullptr : state(j, 0);
      a->ze_c_new = (j == 0) ? nullptr : state(j, 1);
    }
    ea.Tout = w.Tb[cur] + M.offset;
    sa.R = w.Rb[cur] + M.roff;
    sa.S = M.S;
    // non-null plain pointers keep the (unused) plain path well-defined
    ea.nu_c = ea.nu_c_prev; sa.nu_p = sa.nu_p_prev;
    HIP_TRY(launch_cluster_pair<T>(ea, sa, P->cplx, MODE_GIBBS, E ? E->block : 64, s));
  }
  MsgArgs<T> a{};
  a.M = M.M;
  a.comps = M.comps;
  a.S = M.S;
  a.rslot = M.rslot;
  a.inst = M.inst;
  a.R = w.Rb[(n - 1) % 2] + M.roff;
  a.Tm = w.Tb[(n - 1) % 2] + M.offset;
  a.nu = nu;
  a.ze = ze;
  a.nu_src = state(n - 1, 0);
  a.ze_src = state(n - 1, 1);
  a.fp = P->fp + n;
  HIP_TRY(launch_msg<T>(a, MSG_NESTEROV, 256, s));
  return LRH_OK;
}

template <typename T>
lrh_status nesterov_fused(lrh_problem_s* P, T* nu, T* ze, lrh_nesterov_state* stt, int n_iter,
                          hipStream_t s) {
  lrh_status st = ensure_work<T>(P, true);
  if (st != LRH_OK) return st;
  constexpr int CH = kFusedTableMax - 1;  // iterations per captured graph
  const int prec = sizeof(T) == 4 ? 32 : 64;
  int done = 0;
  while (done < n_iter) {
    const int n = std::min(CH, n_iter - done);
    FusedTable tab{};
    double th = stt->theta, thp = 0.0;
    for (int j = 0; j <= n; ++j) {
      FusedParams& f = tab.p[j];
      f.theta_prev = thp;
      f.inv_thL_prev = j > 0 ? 1.0 / (thp * stt->L) : 0.0;
      f.theta_cur = th;
      f.beta = stt->beta;
      thp = th;
      th = theta_next(th);
    }
    HIP_TRY(launch_set_fused(P->fp, tab, n + 1, s));
    if (n == CH) {
      lrh_status gst = launch_cached_graph(P, GraphKey{prec, nu, ze, P->settings_gen}, s, [&](hipStream_t cs) {
        return fused_enqueue<T>(P, nu, ze, n, cs);
      });
      if (gst != LRH_OK) return gst;
    } else {
      if ((st = fused_enqueue<T>(P, nu, ze, n, s)) != LRH_OK) return st;
    }
    for (int j = 0; j < n; ++j) stt->theta = theta_next(stt->theta);
    stt->k += n;
    done += n;
  }
  return LRH_OK;
}

// Plain iterations driven from the device parameter table (row j: theta_k, 1/(theta_k L), beta),
// so that a chunk can be captured once and replayed for any stage.
template <typename T>
lrh_status table_enqueue(lrh_problem_s* P, T* nu, T* ze, int n, hipStream_t s) {
  lrh_status st;
  for (int j = 0; j < n; ++j) {
    if ((st = cluster_pass<T>(P, nu, ze, 0.0, MODE_GIBBS, 0.0, nullptr, s, P->fp + j)) != LRH_OK) return st;
    for (const MBucket& M : P->mb) {
      MsgArgs<T> a = msg_args<T>(P, M);
      a.nu = nu + M.offset;
      a.ze = ze + M.offset;
      a.fp = P->fp + j;
      a.fp_cur = 1;
      HIP_TRY(launch_msg<T>(a, MSG_NESTEROV, 256, s));
    }
  }
  return LRH_OK;
}

template <typename T>
lrh_status nesterov_graph(lrh_problem_s* P, T* nu, T* ze, lrh_nesterov_state* stt, int n_iter, hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  constexpr int CH = kFusedTableMax - 1;
  const int prec = (sizeof(T) == 4 ? 32 : 64) + 1000;  // distinct key space from the fused graphs
  int done = 0;
  while (done < n_iter) {
    const int n = std::min(CH, n_iter - done);
    FusedTable tab{};
    double th = stt->theta;
    for (int j = 0; j < n; ++j) {
      tab.p[j].theta_cur = th;
      tab.p[j].inv_thL_cur = 1.0 / (th * stt->L);
      tab.p[j].beta = stt->beta;
      th = theta_next(th);
    }
    HIP_TRY(launch_set_fused(P->fp, tab, n, s));
    if (n == CH) {
      lrh_status gst = launch_cached_graph(P, GraphKey{prec, nu, ze, P->settings_gen}, s, [&](hipStream_t cs) {
        return table_enqueue<T>(P, nu, ze, n, cs);
      });
      if (gst != LRH_OK) return gst;
    } else {
      if ((st = table_enqueue<T>(P, nu, ze, n, s)) != LRH_OK) return st;
    }
    for (int j = 0; j < n; ++j) stt->theta = theta_next(stt->theta);
    stt->k += n;
    done += n;
  }
  return LRH_OK;
}

template <typename T>
lrh_status nesterov_t(lrh_problem_s* P, T* nu, T* ze, lrh_nesterov_state* stt, int n_iter, bool fused,
                      hipStream_t s) {
  if (stt->k == 0) {
    HIP_TRY(launch_copy<T>(ze, nu, P->nu_len, s));
    stt->theta = 1.0;
  }
  if (n_iter == 0) return LRH_OK;
  if (fused) {
    if (fusable(P)) return nesterov_fused<T>(P, nu, ze, stt, n_iter, s);
    return nesterov_graph<T>(P, nu, ze, stt, n_iter, s);
  }
  return nesterov_plain<T>(P, nu, ze, stt, n_iter, s);
}


// ------------------------------------------------------------------------------------------
// adjoint drivers
// ------------------------------------------------------------------------------------------

lrh_status ensure_adjoint(lrh_problem_s* P) {
  lrh_status st = ensure_work<double>(P, false);
  if (st != LRH_OK) return st;
  if (!P->ywork) {
    if ((st = P->dalloc(&P->ywork, std::max<int64_t>(P->marg_len, 1))) != LRH_OK) return st;
    if ((st = P->dalloc(&P->ones, std::max<int64_t>(P->n_inst, 1))) != LRH_OK) return st;
    std::vector<double> one(std::max<int64_t>(P->n_inst, 1), 1.0);
    HIP_TRY(hipMemcpy(P->ones, one.data(), one.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  return LRH_OK;
}

// One VJP pass over every cluster: Y_e into the marginal slots, the partial traces and ywork.
lrh_status vjp_pass(lrh_problem_s* P, const double* nu, double beta, const double* qbar, const double* gbar,
                    double gb_offscale, hipStream_t s) {
  Work<double>& w = P->w64;
  for (const CBucket& B : P->cb) {
    ClusterArgs<double> a = base_args<double>(P, B);
    a.tol = P->tol_override > 0 ? P->tol_override : default_tol<double>();
    if (B.mb_child >= 0) {
      const MBucket& M = P->mb[B.mb_child];
      a.nu_c = nu + M.offset;
      a.gb_c = gbar ? gbar + M.offset : nullptr;
      a.Tout = w.Tb[0] + M.offset;
    }
    if (B.mb_self >= 0) {
      const MBucket& M = P->mb[B.mb_self];
      a.nu_p = nu + M.offset;
      a.gb_p = gbar ? gbar + M.offset : nullptr;
      a.R = w.Rb[0] + M.roff;
    }
    a.gb_offscale = gb_offscale;
    a.qbar = qbar;
    a.cinst = P->cinst;
    a.marg = P->ywork;
    a.marg_off = P->marg_off;
    a.beta = beta;
    hipError_t e = launch_cluster_vjp(a, P->cplx, beta > 0 ? MODE_GIBBS : MODE_GROUND, s);
    if (e == hipErrorInvalidValue) return fail(LRH_E_UNSUPPORTED, "adjoint of complex clusters with D_e = 64 or of D_e > 64");
    HIP_TRY(e);
  }
  return LRH_OK;
}

lrh_status scatter_grad(lrh_problem_s* P, double* out, hipStream_t s) {
  for (const MBucket& M : P->mb) {
    MsgArgs<double> a = msg_args<double>(P, M);
    a.grad = out + M.offset;
    HIP_TRY(launch_msg<double>(a, MSG_GRAD, 256, s));
  }
  return LRH_OK;
}

lrh_status to_packed(lrh_problem_s* P, double* x, hipStream_t s) {
  for (const MBucket& M : P->mb) HIP_TRY(launch_scale_offdiag(x + M.offset, M.M, M.D, P->cplx, 2.0, s));
  return LRH_OK;
}

lrh_status param_bar(lrh_problem_s* P, double* out, int accumulate, hipStream_t s) {
  if (!out || P->n_params == 0) return LRH_OK;
  HIP_TRY(launch_param_bar(out, accumulate, P->n_params, P->pp_ptr, P->pp_yoff, P->pp_doff, P->pp_D, P->ywork,
                           P->dterm, P->cplx, s));
  return LRH_OK;
}

lrh_status unrolled_grad(lrh_problem_s* P, const double* nu0, double beta, double L, int T, const double* qbar,
                         double* bound, double* pbar, double* nu0bar, bool packed, hipStream_t s) {
  lrh_status st = ensure_adjoint(P);
  if (st != LRH_OK) return st;
  const int64_t n = std::max<int64_t>(P->nu_len, 1);
  const int64_t need = 7 + (int64_t)T;
  if ((int64_t)P->adj_ws.size() < need) {
    for (int64_t i = (int64_t)P->adj_ws.size(); i < need; ++i) {
      double* b = nullptr;
      if ((st = P->dalloc(&b, n)) != LRH_OK) return st;
      P->adj_ws.push_back(b);
    }
  }
  double* nu = P->adj_ws[0];
  double* ze = P->adj_ws[1];
  double* a = P->adj_ws[2];
  double* b = P->adj_ws[3];
  double* btot = P->adj_ws[4];
  double* gb = P->adj_ws[5];
  double* eb = P->adj_ws[6];
  auto eta = [&](int k) { return P->adj_ws[7 + k]; };
  if (nu0) HIP_TRY(launch_copy<double>(nu, nu0, P->nu_len, s));
  else HIP_TRY(hipMemsetAsync(nu, 0, n * sizeof(double), s));
  HIP_TRY(launch_copy<double>(ze, nu, P->nu_len, s));
  std::vector<double> ths;
  double th = 1.0;
  for (int k = 0; k < T; ++k) {
    HIP_TRY(launch_extrap<double>(eta(k), nu, ze, th, P->nu_len, s));
    if ((st = cluster_pass<double>(P, eta(k), nullptr, 0.0, MODE_GIBBS, beta, nullptr, s)) != LRH_OK) return st;
    for (const MBucket& M : P->mb) {
      MsgArgs<double> m = msg_args<double>(P, M);
      m.nu = nu + M.offset;
      m.ze = ze + M.offset;
      m.theta = th;
      m.inv_thL = 1.0 / (th * L);
      HIP_TRY(launch_msg<double>(m, MSG_NESTEROV, 256, s));
    }
    ths.push_back(th);
    th = theta_next(th);
  }
  // B_T = Q(nu^T) and its cotangent
  if ((st = cluster_pass<double>(P, nu, nullptr, 0.0, MODE_GROUND, 0.0, nullptr, s)) != LRH_OK) return st;
  HIP_TRY(launch_reduce(P->scal, P->inst_ptr, P->n_inst, bound, nullptr, nullptr, nullptr, nullptr, nullptr, s));
  const double* qb = qbar ? qbar : P->ones;
  if ((st = vjp_pass(P, nu, 0.0, qb, nullptr, 1.0, s)) != LRH_OK) return st;
  if ((st = scatter_grad(P, a, s)) != LRH_OK) return st;
  if ((st = param_bar(P, pbar, 0, s)) != LRH_OK) return st;
  HIP_TRY(hipMemsetAsync(b, 0, n * sizeof(double), s));
  for (int k = T - 1; k >= 0; --k) {
    const double t = ths[k];
    HIP_TRY(launch_adj_pre(a, b, btot, gb, t, 1.0 / (t * L), P->nu_len, s));
    if ((st = vjp_pass(P, eta(k), beta, nullptr, gb, 1.0, s)) != LRH_OK) return st;
    if ((st = scatter_grad(P, eb, s)) != LRH_OK) return st;
    if ((st = param_bar(P, pbar, 1, s)) != LRH_OK) return st;
    HIP_TRY(launch_adj_post(a, b, btot, eb, t, P->nu_len, s));
  }
  if (nu0bar) {
    HIP_TRY(launch_adj_pre(a, b, nu0bar, gb, 1.0, 0.0, P->nu_len, s));  // nu0_bar = a + b
    if (packed && (st = to_packed(P, nu0bar, s)) != LRH_OK) return st;
  }
  return LRH_OK;
}

// ------------------------------------------------------------------------------------------
// autotuner: per cluster bucket, the launch shape (threads per block of the register kernels,
// lanes per cluster of the LDS kernels) with the shortest measured Gibbs pass
// ------------------------------------------------------------------------------------------

std::string shape_key(const CBucket& B, bool cplx, int prec) {
  return std::to_string(B.De) + "," + std::to_string(B.Dc) + "," + (cplx ? "c" : "r") + "," +
         std::to_string(prec) + "," + std::to_string(B.n);
}

void read_cache(const char* path, std::map<std::string, std::pair<int, int>>& out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[128];
    int block = 0, W = 0;
    // line format:   "De,Dc,kind,prec,n": {"block": B, "W": W, ...
    if (std::sscanf(line, " \"%127[^\"]\": {\"block\": %d, \"W\": %d", key, &block, &W) == 3) out[key] = {block, W};
  }
  std::fclose(f);
}

void write_cache(const char* path, const std::map<std::string, std::tuple<int, int, double>>& rows) {
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : rows) {
    std::fprintf(f, "  \"%s\": {\"block\": %d, \"W\": %d, \"us\": %.3f}%s\n", kv.first.c_str(), std::get<0>(kv.second),
                 std::get<1>(kv.second), std::get<2>(kv.second), ++i < rows.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

template <typename T>
lrh_status autotune_t(lrh_problem_s* P, const char* cache, hipStream_t s) {
  lrh_status st = ensure_work<T>(P, false);
  if (st != LRH_OK) return st;
  const int prec = sizeof(T) == 4 ? 32 : 64;
  std::map<std::string, std::pair<int, int>> cached;
  if (cache) read_cache(cache, cached);
  // non-trivial seeded messages, so every candidate runs full Jacobi sweeps
  T* z = nullptr;
  if ((st = P->dalloc(&z, std::max<int64_t>(P->nu_len, 1))) != LRH_OK) return st;
  HIP_TRY(launch_fill_noise<T>(z, P->nu_len, 0.3, 12345u, s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  Work<T>& w = P->work<T>();
  std::map<std::string, std::tuple<int, int, double>> rows;
  for (CBucket& B : P->cb) {
    const std::string key = shape_key(B, P->cplx, prec);
    const bool dbl = sizeof(T) == 8;
    int& Wsel = dbl ? B.W64 : B.W;
    auto it = cached.find(key);
    if (it != cached.end()) {
      B.block = it->second.first;
      Wsel = it->second.second;
      rows[key] = std::make_tuple(B.block, Wsel, 0.0);
      continue;
    }
    std::vector<std::pair<int, int>> cands;
    {
      int shapes[8];
      const int ns = cluster_shapes(B.De, B.Dc, dbl, P->cplx, MODE_GIBBS, shapes);
      const bool has_expm = std::find(shapes, shapes + ns, 0) != shapes + ns ||
                            std::find(shapes, shapes + ns, 4) != shapes + ns;
      for (int i = 0; i < ns; ++i) {
        if (has_expm && B.De >= 128 && shapes[i] != 0 && shapes[i] != 4) continue;  // slab Jacobi: far slower
        if (shapes[i] == 1 || B.De <= 4)
          for (int b : {64, 128, 256}) cands.push_back({b, shapes[i]});
        else
          cands.push_back({B.block, shapes[i]});
      }
    }
    double best = 1e30;
    std::pair<int, int> pick = cands[0];
    for (auto& cand : cands) {
      ClusterArgs<T> a = base_args<T>(P, B);
      if (B.mb_child >= 0) {
        const MBucket& M = P->mb[B.mb_child];
        a.nu_c = z + M.offset;
        a.Tout = w.Tb[0] + M.offset;
      }
      if (B.mb_self >= 0) {
        const MBucket& M = P->mb[B.mb_self];
        a.nu_p = z + M.offset;
        a.R = w.Rb[0] + M.roff;
      }
      a.beta = 1.0;
      HIP_TRY(hipEventRecord(e0, s));
      HIP_TRY(launch_cluster<T>(a, P->cplx, MODE_GIBBS, cand.first, cand.second, s));  // warm-up
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms0 = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms0, e0, e1));
      if (1e3 * ms0 > 4.0 * best) continue;   // clearly slower than the best so far
      const int reps = B.n > 100000 ? 3 : 10;
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) HIP_TRY(launch_cluster<T>(a, P->cplx, MODE_GIBBS, cand.first, cand.second, s));
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1e3 * ms / reps;
      if (us < best) {
        best = us;
        pick = cand;
      }
    }
    B.block = pick.first;
    Wsel = pick.second;
    B.tuned_us = best;
    rows[key] = std::make_tuple(B.block, Wsel, best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (cache) write_cache(cache, rows);
  return LRH_OK;
}
}  // namespace

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------

extern "C" {

const char* lrh_last_error(void) { return g_err.c_str(); }

const char* lrh_build_info(void) {
  static const std::string info = "HIP headers " + std::to_string(HIP_VERSION_MAJOR) + "." +
                                  std::to_string(HIP_VERSION_MINOR) + "." + std::to_string(HIP_VERSION_PATCH) +
                                  ", device code gfx950";
  return info.c_str();
}

lrh_status lrh_build_clusters(const lrh_problem_desc* desc, int hip_device, lrh_problem* out) {
  if (!out) return fail(LRH_E_INVALID, "null output handle");
  *out = nullptr;
  std::unique_ptr<lrh_problem_s> P(new lrh_problem_s());
  lrh_status st;
  if (hip_device < 0) {
    P->host_only = true;
    try {
      st = build(desc, P.get());
    } catch (const std::bad_alloc&) {
      return fail(LRH_E_NOMEM, "host allocation failed");
    }
  } else {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device >= ndev) return fail(LRH_E_DEVICE, "invalid HIP device");
    DeviceGuard guard(hip_device);
    P->device = hip_device;
    try {
      st = build(desc, P.get());
    } catch (const std::bad_alloc&) {
      return fail(LRH_E_NOMEM, "host allocation failed");
    }
    if (st == LRH_OK) bind_static_scratch(hip_device);   // the device is current here
  }
  if (st != LRH_OK) return st;
  *out = P.release();
  return LRH_OK;
}

lrh_status lrh_query(lrh_problem p, lrh_layout* out) {
  if (!p || !out) return fail(LRH_E_INVALID, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->n_clusters = p->n_clusters;
  out->n_msgs = p->n_msgs;
  out->n_instances = p->n_inst;
  out->is_real = p->cplx ? 0 : 1;
  out->max_D = p->max_D;
  out->n_buckets = (int32_t)p->mb.size();
  for (size_t b = 0; b < p->mb.size(); ++b) {
    out->bucket_D[b] = p->mb[b].D;
    out->bucket_count[b] = p->mb[b].M;
    out->bucket_comps[b] = p->mb[b].comps;
    out->bucket_offset[b] = p->mb[b].offset;
  }
  out->nu_len = p->nu_len;
  out->marg_len = p->marg_len;
  out->Lambda_G = p->Lambda;
  out->Gamma_G = p->Gamma;
  out->max_sweeps = p->max_sweeps;
  out->n_params = (int32_t)p->n_params;
  return LRH_OK;
}

lrh_status lrh_export_clusters(lrh_problem p, int64_t* ptr, int32_t* sites, int32_t* instance) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (ptr) std::memcpy(ptr, p->c_ptr.data(), p->c_ptr.size() * sizeof(int64_t));
  if (sites) std::memcpy(sites, p->c_sites.data(), p->c_sites.size() * sizeof(int32_t));
  if (instance) std::memcpy(instance, p->c_inst.data(), p->c_inst.size() * sizeof(int32_t));
  return LRH_OK;
}

lrh_status lrh_export_messages(lrh_problem p, int32_t* parent, int32_t* child, int32_t* bucket,
                               int64_t* index) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  const size_t n = p->m_parent.size();
  if (parent) std::memcpy(parent, p->m_parent.data(), n * sizeof(int32_t));
  if (child) std::memcpy(child, p->m_child.data(), n * sizeof(int32_t));
  if (bucket) std::memcpy(bucket, p->m_bucket.data(), n * sizeof(int32_t));
  if (index) std::memcpy(index, p->m_index.data(), n * sizeof(int64_t));
  return LRH_OK;
}

lrh_status lrh_dual_eval(lrh_problem p, const void* nu, uint32_t flags, double beta, double* q_dev,
                         void* grad_dev, void* marg_dev, hipStream_t stream) {
  if (!p || !nu || !q_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(beta >= 0.0)) return fail(LRH_E_INVALID, "beta must be >= 0");
  DeviceGuard guard(p->device);
  if (flags & LRH_F32)
    return dual_eval_t<float>(p, (const float*)nu, beta, q_dev, (float*)grad_dev, (float*)marg_dev, stream);
  return dual_eval_t<double>(p, (const double*)nu, beta, q_dev, (double*)grad_dev, (double*)marg_dev, stream);
}

lrh_status lrh_step_subgrad(lrh_problem p, void* nu, void* nu_best, double* q_best_dev, int64_t k0,
                            int32_t n_iter, int32_t step_kind, double step_scale, double* q_hist_dev,
                            uint32_t flags, hipStream_t stream) {
  if (!p || !nu || !nu_best || !q_best_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (n_iter < 0 || k0 < 0) return fail(LRH_E_INVALID, "negative iteration counts");
  if (!(step_scale > 0.0) || (step_kind != 0 && step_kind != 1)) return fail(LRH_E_INVALID, "bad step rule");
  DeviceGuard guard(p->device);
  if (flags & LRH_F32)
    return subgrad_t<float>(p, (float*)nu, (float*)nu_best, q_best_dev, k0, n_iter, step_kind, step_scale,
                            q_hist_dev, stream);
  return subgrad_t<double>(p, (double*)nu, (double*)nu_best, q_best_dev, k0, n_iter, step_kind, step_scale,
                           q_hist_dev, stream);
}

lrh_status lrh_step_nesterov(lrh_problem p, void* nu, void* zeta, lrh_nesterov_state* st, int32_t n_iter,
                             uint32_t flags, hipStream_t stream) {
  if (!p || !nu || !zeta || !st) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(st->beta > 0.0) || !std::isfinite(st->beta)) return fail(LRH_E_INVALID, "beta must be positive and finite");
  if (!(st->L >= 0.0) || !std::isfinite(st->L)) return fail(LRH_E_INVALID, "L must be >= 0 and finite");
  if (st->L == 0.0) st->L = st->beta * p->Lambda / 2.0;   // the paper's L_beta = beta Lambda_G / 2
  if (n_iter < 0 || st->k < 0) return fail(LRH_E_INVALID, "negative iteration counts");
  if (st->k > 0 && !(st->theta > 0.0 && st->theta <= 1.0)) return fail(LRH_E_INVALID, "theta out of (0, 1]");
  DeviceGuard guard(p->device);
  const bool fused = (flags & LRH_FUSED) != 0;
  if (flags & LRH_F32) return nesterov_t<float>(p, (float*)nu, (float*)zeta, st, n_iter, fused, stream);
  return nesterov_t<double>(p, (double*)nu, (double*)zeta, st, n_iter, fused, stream);
}

lrh_status lrh_certify(lrh_problem p, const void* nu, uint32_t flags, double* q_dev, double* margin_dev,
                       double* lmin_dev, hipStream_t stream) {
  if (!p || !nu || !q_dev || !margin_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  DeviceGuard guard(p->device);
  {
    lrh_status wst = ensure_work<double>(p, false);
    if (wst != LRH_OK) return wst;
  }
  const double* nu64 = (const double*)nu;
  if (flags & LRH_F32) {
    if (!p->nu64_tmp) {
      lrh_status st = p->dalloc(&p->nu64_tmp, std::max<int64_t>(p->nu_len, 1));
      if (st != LRH_OK) return st;
    }
    HIP_TRY(launch_widen(p->nu64_tmp, (const float*)nu, p->nu_len, stream));
    nu64 = p->nu64_tmp;
  }
  const int64_t wsl = cert_ws_len(p);
  if (wsl > 0 && !p->cert_ws) {
    lrh_status st = p->dalloc(&p->cert_ws, wsl);
    if (st != LRH_OK) return st;
  }
  for (const CBucket& B : p->cb) {
    ClusterArgs<double> a = base_args<double>(p, B);
    a.tol = default_tol<double>();   // certification ignores a loosened iteration tolerance
    a.cert_ws = p->cert_ws;
    if (B.mb_child >= 0) a.nu_c = nu64 + p->mb[B.mb_child].offset;
    if (B.mb_self >= 0) a.nu_p = nu64 + p->mb[B.mb_self].offset;
    a.R = nullptr;
    HIP_TRY(launch_cluster<double>(a, p->cplx, MODE_CERTIFY, B.block, shape_for(p, B, true, MODE_CERTIFY), stream));
  }
  HIP_TRY(launch_reduce(p->scal, p->inst_ptr, p->n_inst, q_dev, p->scal2, margin_dev, nullptr, nullptr, nullptr,
                        stream));
  if (lmin_dev) HIP_TRY(launch_copy<double>(lmin_dev, p->scal, p->n_clusters, stream));
  return LRH_OK;
}

lrh_status lrh_certify_noalloc(lrh_problem p, const void* nu, uint32_t flags, double* q_dev, double* margin_dev,
                               double* lmin_dev, hipStream_t stream) {
  if (!p || !nu || !q_dev || !margin_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  DeviceGuard guard(p->device);
  std::string why;
  unsigned char* base = (unsigned char*)static_scratch(p->device, why);
  if (!base) return fail(LRH_E_DEVICE, why);
  // layout of the static array: [widened messages (LRH_F32 only)][tridiagonalisation slabs]
  size_t off = 0;
  const double* nu64 = (const double*)nu;
  if (flags & LRH_F32) {
    const size_t need = ((size_t)std::max<int64_t>(p->nu_len, 1) * sizeof(double) + 255) / 256 * 256;
    if (need > kStaticScratchBytes)
      return fail(LRH_E_UNSUPPORTED, "float messages need " + std::to_string(need) +
                                         " bytes widened, beyond the static workspace of " +
                                         std::to_string(kStaticScratchBytes));
    HIP_TRY(launch_widen((double*)base, (const float*)nu, p->nu_len, stream));
    nu64 = (const double*)base;
    off = need;
  }
  // one slab (the matrix, real and imaginary planes) per workgroup of the tridiagonalisation
  // kernel (D_e >= 64); fewer slabs than clusters: each workgroup takes several in turn
  int Dmax = 0;
  int64_t nwg = 0;
  for (const CBucket& B : p->cb)
    if (B.De >= 64 && shape_for(p, B, true, MODE_CERTIFY) == 2) {
      Dmax = std::max(Dmax, B.De);
      nwg = std::max<int64_t>(nwg, B.n);
    }
  const int64_t slab = (int64_t)(p->cplx ? 2 : 1) * Dmax * Dmax;
  int64_t blocks = 0;
  if (Dmax > 0) {
    blocks = std::min<int64_t>({nwg, 1024, (int64_t)((kStaticScratchBytes - off) / (slab * sizeof(double)))});
    if (blocks < 1)
      return fail(LRH_E_UNSUPPORTED, "no room for one " + std::to_string(Dmax) + "-dimensional slab in the static workspace");
  }
  // tridiagonals of the 16- and 32-dimensional buckets, after the slabs if they fit (else those
  // buckets use the one-wave kernel, which needs no workspace)
  const size_t slab_bytes = ((size_t)std::max<int64_t>(blocks, 0) * slab * sizeof(double) + 255) / 256 * 256;
  const size_t ws_bytes = (size_t)cert_ws_len(p) * sizeof(double);
  double* ws = (ws_bytes > 0 && off + slab_bytes + ws_bytes <= kStaticScratchBytes)
                   ? (double*)(base + off + slab_bytes) : nullptr;
  for (const CBucket& B : p->cb) {
    ClusterArgs<double> a = base_args<double>(p, B);
    a.tol = default_tol<double>();
    a.big_scratch = nullptr;
    a.big_blocks = 0;
    a.cert_ws = ws;
    a.expm_scratch = Dmax > 0 ? (double*)(base + off) : nullptr;
    a.expm_slab = slab;
    a.expm_blocks = blocks;
    if (B.mb_child >= 0) a.nu_c = nu64 + p->mb[B.mb_child].offset;
    if (B.mb_self >= 0) a.nu_p = nu64 + p->mb[B.mb_self].offset;
    a.R = nullptr;
    HIP_TRY(launch_cluster<double>(a, p->cplx, MODE_CERTIFY, B.block, shape_for(p, B, true, MODE_CERTIFY), stream));
  }
  HIP_TRY(launch_reduce(p->scal, p->inst_ptr, p->n_inst, q_dev, p->scal2, margin_dev, nullptr, nullptr, nullptr,
                        stream));
  if (lmin_dev) HIP_TRY(launch_copy<double>(lmin_dev, p->scal, p->n_clusters, stream));
  return LRH_OK;
}

lrh_status lrh_set_params(lrh_problem p, const double* params_dev, hipStream_t stream) {
  if (!p || !params_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (p->n_params == 0) return fail(LRH_E_INVALID, "problem has no parameters");
  DeviceGuard guard(p->device);
  HIP_TRY(launch_set_params(p->h, p->hfix, p->pc_hoff, p->pc_ptr, p->pc_param, p->pc_doff, p->dterm, p->pc_ncomp,
                            p->n_pc, params_dev, stream));
  return LRH_OK;
}

lrh_status lrh_dual_vjp(lrh_problem p, const void* nu, uint32_t flags, double beta, const double* qbar_dev,
                        const void* gbar_dev, void* nu_bar_dev, double* param_bar_dev, hipStream_t stream) {
  if (!p || !nu) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(beta >= 0.0)) return fail(LRH_E_INVALID, "beta must be >= 0");
  if (beta == 0.0 && gbar_dev) return fail(LRH_E_INVALID, "the subgradient has no derivative (gbar with beta = 0)");
  if (flags & LRH_F32) return fail(LRH_E_UNSUPPORTED, "the adjoint runs in FP64 only");
  DeviceGuard guard(p->device);
  lrh_status st = ensure_adjoint(p);
  if (st != LRH_OK) return st;
  const bool packed = (flags & LRH_PACKED_COTANGENT) != 0;
  if ((st = vjp_pass(p, (const double*)nu, beta, qbar_dev, (const double*)gbar_dev, packed ? 0.5 : 1.0, stream)) !=
      LRH_OK)
    return st;
  if (nu_bar_dev) {
    if ((st = scatter_grad(p, (double*)nu_bar_dev, stream)) != LRH_OK) return st;
    if (packed && (st = to_packed(p, (double*)nu_bar_dev, stream)) != LRH_OK) return st;
  }
  return param_bar(p, param_bar_dev, 0, stream);
}

lrh_status lrh_unrolled_bound_grad(lrh_problem p, const double* nu0_dev, double beta, double L, int32_t T,
                                   const double* qbar_dev, double* bound_dev, double* param_bar_dev,
                                   double* nu0_bar_dev, uint32_t flags, hipStream_t stream) {
  if (!p || !bound_dev) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(beta > 0.0) || !(L >= 0.0) || T < 0) return fail(LRH_E_INVALID, "beta > 0, L >= 0 and T >= 0 required");
  if (L == 0.0) L = beta * p->Lambda / 2.0;
  if (flags & LRH_F32) return fail(LRH_E_UNSUPPORTED, "the adjoint runs in FP64 only");
  DeviceGuard guard(p->device);
  return unrolled_grad(p, nu0_dev, beta, L, T, qbar_dev, bound_dev, param_bar_dev, nu0_bar_dev,
                       (flags & LRH_PACKED_COTANGENT) != 0, stream);
}

lrh_status lrh_check(lrh_problem p, hipStream_t stream, int64_t* noconv, int64_t* nonfinite) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  DeviceGuard guard(p->device);
  HIP_TRY(hipStreamSynchronize(stream));
  unsigned long long h[2] = {0, 0};
  HIP_TRY(hipMemcpy(h, p->health, sizeof(h), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(p->health, 0, sizeof(h)));
  if (noconv) *noconv = (int64_t)h[0];
  if (nonfinite) *nonfinite = (int64_t)h[1];
  if (h[1]) return fail(LRH_E_NONFINITE, "non-finite eigenvalue in " + std::to_string(h[1]) + " cluster solves");
  if (h[0]) return fail(LRH_E_NOCONV, "Jacobi sweep cap reached in " + std::to_string(h[0]) + " cluster solves");
  return LRH_OK;
}

lrh_status lrh_certify_fallbacks(lrh_problem p, hipStream_t stream, int64_t* count) {
  if (!p || !count) return fail(LRH_E_INVALID, "null argument");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  DeviceGuard guard(p->device);
  HIP_TRY(hipStreamSynchronize(stream));
  unsigned long long h = 0;
  HIP_TRY(hipMemcpy(&h, p->health + 2, sizeof(h), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(p->health + 2, 0, sizeof(h)));
  *count = (int64_t)h;
  return LRH_OK;
}

lrh_status lrh_set_certify_method(lrh_problem p, int32_t method) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (method < 0 || method > 3) return fail(LRH_E_INVALID, "method must be 0, 1, 2 or 3");
  p->cert_method = method;
  return LRH_OK;
}

lrh_status lrh_autotune(lrh_problem p, uint32_t flags, const char* cache_path, hipStream_t stream) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  DeviceGuard guard(p->device);
  settings_changed(p);
  if (flags & LRH_F32) return autotune_t<float>(p, cache_path, stream);
  return autotune_t<double>(p, cache_path, stream);
}

lrh_status lrh_get_shapes(lrh_problem p, int32_t cap, int32_t* De, int32_t* Dc, int64_t* n, int32_t* block,
                          int32_t* W, double* us, int32_t* count) {
  if (!p || !count) return fail(LRH_E_INVALID, "null argument");
  *count = (int32_t)p->cb.size();
  for (int32_t i = 0; i < std::min<int32_t>(cap, *count); ++i) {
    const CBucket& B = p->cb[i];
    if (De) De[i] = B.De;
    if (Dc) Dc[i] = B.Dc;
    if (n) n[i] = B.n;
    if (block) block[i] = B.block;
    if (W) W[i] = B.W;  // FP32 iteration shape
    if (us) us[i] = B.tuned_us;
  }
  return LRH_OK;
}

lrh_status lrh_set_shape(lrh_problem p, int32_t De, int32_t block, int32_t W, uint32_t flags) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (block != 64 && block != 128 && block != 256) return fail(LRH_E_INVALID, "block must be 64, 128 or 256");
  const bool dbl = !(flags & LRH_F32);
  bool any = false;
  for (CBucket& B : p->cb) {
    if (B.De != De) continue;
    int shapes[8];
    const int n = cluster_shapes(B.De, B.Dc, dbl, p->cplx, MODE_GIBBS, shapes);
    bool ok = false;
    for (int i = 0; i < n; ++i) ok = ok || shapes[i] == W;
    if (!ok) return fail(LRH_E_UNSUPPORTED, "launch shape not compiled for this bucket");
    B.block = block;
    (dbl ? B.W64 : B.W) = W;
    any = true;
  }
  if (!any) return fail(LRH_E_INVALID, "no cluster bucket with that dimension");
  settings_changed(p);
  return LRH_OK;
}

lrh_status lrh_time_buckets(lrh_problem p, const void* nu, uint32_t flags, double beta, int32_t reps, double* us,
                            hipStream_t stream) {
  if (!p || !nu || !us || reps < 1) return fail(LRH_E_INVALID, "null argument or reps < 1");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(LRH_E_INVALID, "beta must be finite and >= 0");
  DeviceGuard guard(p->device);
  if (flags & LRH_F32) return time_buckets_t<float>(p, (const float*)nu, beta, reps, us, stream);
  return time_buckets_t<double>(p, (const double*)nu, beta, reps, us, stream);
}

lrh_status lrh_time_messages(lrh_problem p, void* nu, void* zeta, uint32_t flags, double beta, int32_t reps,
                             double* us, hipStream_t stream) {
  if (!p || !nu || !zeta || !us || reps < 1) return fail(LRH_E_INVALID, "null argument or reps < 1");
  if (p->host_only) return fail(LRH_E_INVALID, "problem was built without a device");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(LRH_E_INVALID, "beta must be finite and > 0");
  DeviceGuard guard(p->device);
  if (flags & LRH_F32) return time_messages_t<float>(p, (float*)nu, (float*)zeta, beta, reps, us, stream);
  return time_messages_t<double>(p, (double*)nu, (double*)zeta, beta, reps, us, stream);
}

lrh_status lrh_set_jacobi(lrh_problem p, int32_t max_sweeps, double rel_tol) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (max_sweeps < 0 || !(rel_tol >= 0.0)) return fail(LRH_E_INVALID, "bad Jacobi settings");
  p->max_sweeps = max_sweeps;
  p->tol_override = rel_tol;
  settings_changed(p);
  return LRH_OK;
}

lrh_status lrh_set_slab_limit(lrh_problem p, int64_t max_slabs) {
  if (!p) return fail(LRH_E_INVALID, "null problem");
  if (max_slabs < 0) return fail(LRH_E_INVALID, "max_slabs must be >= 0");
  p->slab_limit = max_slabs;
  settings_changed(p);
  return LRH_OK;
}

lrh_status lrh_measure_fp64_mfma(int hip_device, double* tflops, hipStream_t stream) {
  if (!tflops) return fail(LRH_E_INVALID, "null argument");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return fail(LRH_E_DEVICE, "invalid HIP device");
  DeviceGuard guard(hip_device);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  const int blocks = 8 * prop.multiProcessorCount;   // 8 waves per SIMD
  const int iters = 4000;
  double* out = nullptr;
  HIP_TRY(hipMalloc(&out, (size_t)blocks * 256 * sizeof(double)));
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err == hipSuccess) err = launch_mfma_f64_rate(out, blocks, iters, stream);   // warm-up
  if (err == hipSuccess) err = hipEventRecord(e0, stream);
  if (err == hipSuccess) err = launch_mfma_f64_rate(out, blocks, iters, stream);
  if (err == hipSuccess) err = hipEventRecord(e1, stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (err != hipSuccess) return fail(LRH_E_DEVICE, std::string("fp64 rate probe: ") + hipGetErrorString(err));
  const double flops = (double)blocks * 4.0 /* waves */ * iters * 8.0 /* chains */ * 2048.0;
  *tflops = flops / (ms * 1e-3) / 1e12;
  return LRH_OK;
}

void lrh_destroy(lrh_problem p) { delete p; }

}  // extern "C"
