// Host planner and C entry points.
//
// ibf_plan builds the dyadic trees of Sec. 3 ("Preliminaries"): T_X on
// [0,1) and T_Omega on the frequency domain, with depth L chosen so that a
// box pair (A at level l, B at level L-l) has w_A * w_B <= 1, and sorts both
// point sets into leaves of about `leaf` points.  Everything here is host
// integer / FP64 bookkeeping; all factor arithmetic runs on the device.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include <atomic>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ibf_internal.h"

namespace {
thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Stable counting sort of points into `nleaf` leaves given their leaf index.
void sort_into_leaves(const std::vector<int64_t>& leaf_of, int64_t nleaf,
                      std::vector<int32_t>& perm, std::vector<int32_t>& off,
                      std::vector<int32_t>& leaf_sorted, int& smax) {
  const int64_t n = (int64_t)leaf_of.size();
  std::vector<int64_t> cnt(nleaf + 1, 0);
  for (int64_t i = 0; i < n; ++i) cnt[leaf_of[i] + 1]++;
  smax = 0;
  for (int64_t b = 0; b < nleaf; ++b) smax = std::max<int64_t>(smax, cnt[b + 1]);
  for (int64_t b = 0; b < nleaf; ++b) cnt[b + 1] += cnt[b];
  off.assign(cnt.begin(), cnt.end());
  perm.assign(n, 0);
  leaf_sorted.assign(n, 0);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i) {
    int64_t b = leaf_of[i];
    perm[pos[b]] = (int32_t)i;
    leaf_sorted[pos[b]] = (int32_t)b;
    pos[b]++;
  }
}
}  // namespace

namespace {
// the installed allocator pair, and the pair that made each live block
std::mutex g_alloc_mu;
ibf_alloc_fn g_alloc = nullptr;
ibf_free_fn g_free = nullptr;
std::unordered_map<void*, ibf_free_fn> g_hooked;
}  // namespace

namespace ibf {
void set_error(const std::string& msg) { g_last_error = msg; }

hipError_t dev_malloc_raw(void** ptr, size_t bytes) {
  ibf_alloc_fn a;
  ibf_free_fn f;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    f = g_free;
  }
  if (!a) return hipMalloc(ptr, bytes);
  void* q = a(bytes, nullptr);
  *ptr = q;
  if (!q) return hipErrorOutOfMemory;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_hooked[q] = f;
  return hipSuccess;
}

hipError_t dev_free(void* ptr) {
  if (!ptr) return hipSuccess;
  ibf_free_fn f = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_hooked.find(ptr);
    if (it != g_hooked.end()) {
      f = it->second;
      g_hooked.erase(it);
    }
  }
  if (!f) return hipFree(ptr);
  // hipFree waits for the device; an allocator's free need not
  const hipError_t e = hipDeviceSynchronize();
  f(ptr, nullptr);
  return e;
}

size_t complex_bytes(int precision) { return precision == IBF_FP64 ? 16 : 8; }

void set_order(ibf_plan_t p, int r, double tol) {
  p->r = r;
  p->geo.r = r;
  p->tol = tol;
  const int L = p->geo.L, l0 = p->geo.l0;
  // Preliminary non-zeros (memory numerator of the compression ratio).
  const int nstages = L - 2 * l0;
  p->nnz_prelim = (p->nx + p->nxi) * ((int64_t)1 << l0) * r +
                  (int64_t)nstages * p->npairs * 2 * r * r + p->npairs * r * r;
  // sweep_in = -1: on iff a leaf holds fewer than r points (Sec. 4.3: the
  // sweep-in is what keeps the ranks of such leaves below r) and no leaf
  // exceeds the sweep-in kernels' 64 points
  if (p->sweep_auto) {
    int32_t mn = INT32_MAX;
    for (size_t b = 0; b + 1 < p->xoff.size(); ++b) mn = std::min(mn, p->xoff[b + 1] - p->xoff[b]);
    for (size_t b = 0; b + 1 < p->xioff.size(); ++b)
      mn = std::min(mn, p->xioff[b + 1] - p->xioff[b]);
    p->sweep_in = (mn < r && p->smax_x <= 64 && p->smax_xi <= 64) ? 1 : 0;
  }
}

void free_factors(ibf_plan_t p) {
  free_adjoint(p);
  for (auto& st : p->stages) {
    if (st.blk) (void)ibf::dev_free(st.blk);
    if (st.qblk) (void)ibf::dev_free(st.qblk);
  }
  p->stages.clear();
  void** bufs[] = {&p->d_vbar, &p->d_ubar, &p->d_mdot, &p->d_work[0], &p->d_work[1],
                   reinterpret_cast<void**>(&p->d_prank)};
  for (void** b : bufs) {
    if (*b) (void)ibf::dev_free(*b);
    *b = nullptr;
  }
  p->work_bytes = 0;
  p->built = false;
}
}  // namespace ibf

extern "C" {

const char* ibf_last_error(void) { return g_last_error.c_str(); }

int ibf_plan(const ibf_desc* d, ibf_plan_t* out) {
  if (!d || !out) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: null argument");
  *out = nullptr;
  if (d->dim != 1 && d->dim != 2)
    return fail(IBF_ERR_UNSUPPORTED, "ibf_plan: dim must be 1 or 2");
  if (d->n_x < 1 || d->n_xi < 1) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: empty point set");
  if (d->n_x > (int64_t)1 << 30 || d->n_xi > (int64_t)1 << 30)
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: more than 2^30 points");
  if (!d->x || !d->xi) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: null point array");
  if (d->dim == 2) return ibf::plan2d(d, out);
  const bool learned = d->r <= 0;
  if (!learned && d->r < 2) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: r must be >= 2");
  if (d->r > ibf::kMaxR) return fail(IBF_ERR_UNSUPPORTED, "ibf_plan: r > 16 not supported");
  if (learned && d->predictor && d->predictor_hidden != 8 && d->predictor_hidden != 16 &&
      d->predictor_hidden != 32)
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: predictor_hidden must be 8, 16 or 32");
  if (!(d->tol > 0.0 && d->tol < 1.0))
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: tol must lie in (0, 1)");
  if (d->leaf < 2 || (d->leaf & (d->leaf - 1)))
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: leaf must be a power of two >= 2");
  if (d->precision < IBF_FP64 || d->precision > IBF_BF16X2)
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: unknown precision");
  if (d->sweep_in < -1 || d->sweep_in > 1)
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: sweep_in must be -1, 0 or 1");
  if (d->svd_samples < 0) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: svd_samples < 0");
  if (d->svd_samples > 0)
    return fail(IBF_ERR_UNSUPPORTED,
                "ibf_plan: the sampled low-rank approximation is provided for dim 2 (the 1-D "
                "blocks have at most 32 columns)");

  ibf::PhaseDesc ph{};
  ph.kind = d->phase_id;
  const double* pp = d->phase_params;
  int np = d->n_params;
  if (np < 0 || np > ibf::kMaxParams || (np > 0 && !pp))
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: bad phase parameters");
  switch (d->phase_id) {
    case IBF_PHASE_DFT:
      ph.p[0] = np >= 1 ? pp[0] : 1.0;
      if (ph.p[0] != 1.0 && ph.p[0] != -1.0)
        return fail(IBF_ERR_INVALID_ARG, "ibf_plan: DFT sign must be +1 or -1");
      break;
    case IBF_PHASE_FIO1D:
      ph.p[0] = np >= 1 ? pp[0] : 2.0;
      ph.p[1] = np >= 2 ? pp[1] : 1.0;
      ph.p[2] = np >= 3 ? pp[2] : 8.0;
      if (ph.p[2] == 0.0) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: p2 == 0");
      break;
    case IBF_PHASE_SEPARABLE:
      ph.p[0] = np >= 1 ? pp[0] : 3.0;
      ph.p[1] = np >= 2 ? pp[1] : 0.3125;
      break;
    default:
      return fail(IBF_ERR_UNSUPPORTED, "ibf_plan: unsupported phase for dim 1");
  }
  // amplitude a(x, xi) of eqn:FIO
  ph.amp = d->amp_id;
  {
    const int na = d->n_amp_params;
    const double* q = d->amp_params;
    if (na < 0 || na > ibf::kMaxParams || (na > 0 && !q))
      return fail(IBF_ERR_INVALID_ARG, "ibf_plan: bad amplitude parameters");
    switch (d->amp_id) {
      case IBF_AMP_NONE:
        break;
      case IBF_AMP_SEPARABLE:
        if (na != 6 || q[5] == 0.0)
          return fail(IBF_ERR_INVALID_ARG, "ibf_plan: separable amplitude takes 6 parameters, q5 != 0");
        for (int i = 0; i < 6; ++i) ph.q[i] = q[i];
        break;
      case IBF_AMP_WAVE:
        if (na != 3 || q[2] == 0.0)
          return fail(IBF_ERR_INVALID_ARG, "ibf_plan: wave amplitude takes 3 parameters, q2 != 0");
        for (int i = 0; i < 3; ++i) ph.q[i] = q[i];
        break;
      default:
        return fail(IBF_ERR_UNSUPPORTED, "ibf_plan: unknown amplitude");
    }
    for (int i = 0; i < na; ++i)
      if (!std::isfinite(q[i])) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: amplitude parameter not finite");
  }

  const double W = d->omega_width > 0 ? d->omega_width : (double)d->n_xi;
  const double lo = d->omega_lo;
  int L = (int)std::ceil(std::log2(W) - 1e-12);
  int l0 = 0;
  while ((1 << l0) < d->leaf) ++l0;
  if (L < 2 * l0)
    return fail(IBF_ERR_INVALID_ARG, "ibf_plan: need omega_width >= leaf^2 (N >= leaf^2)");
  if (L > 30) return fail(IBF_ERR_INVALID_ARG, "ibf_plan: tree too deep");

  auto p = new ibf_plan_s();
  p->dim = 1;
  p->nx = d->n_x;
  p->nxi = d->n_xi;
  p->device = d->device;
  p->phase = ph;
  p->r = d->r;
  p->leaf = d->leaf;
  p->precision = d->precision;
  p->sweep_in = d->sweep_in > 0 ? 1 : 0;
  p->sweep_auto = d->sweep_in < 0 ? 1 : 0;
  p->tol = d->tol;
  p->learned = learned;
  p->predictor = d->predictor;
  p->predictor_hidden = d->predictor_hidden;
  p->target_tol = d->tol;
  if (learned) p->r = 0;
  p->geo = ibf::Geo{L, l0, L / 2, p->r, lo, W};
  if (d->fixed_ranks) {
    p->caps.assign(d->fixed_ranks, d->fixed_ranks + (L - 2 * l0 + 1));
    for (int& c : p->caps) c = std::max(c, 0);
  }
  p->npairs = (int64_t)1 << L;
  p->nleaf = (int64_t)1 << (L - l0);

  // Leaf index of every point: floor(position * 2^(L-l0) / width).
  const int64_t nl = p->nleaf;
  std::vector<int64_t> lx(d->n_x), lxi(d->n_xi);
  for (int64_t i = 0; i < d->n_x; ++i) {
    double v = d->x[i];
    if (!(v >= 0.0 && v < 1.0)) {
      delete p;
      return fail(IBF_ERR_INVALID_ARG, "ibf_plan: x outside [0, 1)");
    }
    int64_t b = (int64_t)std::floor(v * (double)nl);
    lx[i] = std::min<int64_t>(std::max<int64_t>(b, 0), nl - 1);
  }
  for (int64_t j = 0; j < d->n_xi; ++j) {
    double v = d->xi[j];
    if (!(v >= lo && v < lo + W)) {
      delete p;
      return fail(IBF_ERR_INVALID_ARG, "ibf_plan: xi outside the Omega domain");
    }
    int64_t b = (int64_t)std::floor((v - lo) * (double)nl / W);
    lxi[j] = std::min<int64_t>(std::max<int64_t>(b, 0), nl - 1);
  }
  sort_into_leaves(lx, nl, p->perm_x, p->xoff, p->xleaf, p->smax_x);
  sort_into_leaves(lxi, nl, p->perm_xi, p->xioff, p->xileaf, p->smax_xi);
  p->xs.resize(d->n_x);
  p->xis.resize(d->n_xi);
  for (int64_t i = 0; i < d->n_x; ++i) p->xs[i] = d->x[p->perm_x[i]];
  for (int64_t j = 0; j < d->n_xi; ++j) p->xis[j] = d->xi[p->perm_xi[j]];

  if (!learned) ibf::set_order(p, p->r, p->tol);
  *out = p;
  return IBF_OK;
}

int ibf_build(ibf_plan_t p, void* stream) {
  if (!p) return fail(IBF_ERR_INVALID_ARG, "ibf_build: null plan");
  auto t0 = std::chrono::steady_clock::now();
  int rc = p->dim == 2 ? ibf::build2d(p, (hipStream_t)stream)
                       : ibf::build_plan(p, (hipStream_t)stream);
  auto t1 = std::chrono::steady_clock::now();
  p->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  return rc;
}

int ibf_build_batch(ibf_plan_t* plans, int count, int nthreads, void* stream, int* failed) {
  if (failed) *failed = -1;
  if (!plans || count < 1) return fail(IBF_ERR_INVALID_ARG, "ibf_build_batch: no plans");
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return fail(IBF_ERR_INVALID_ARG, "ibf_build_batch: null plan");
  const int dev = plans[0]->device;
  for (int i = 1; i < count; ++i)
    if (plans[i]->device != dev)
      return fail(IBF_ERR_INVALID_ARG, "ibf_build_batch: plans on different devices");
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (plans[i] == plans[j]) return fail(IBF_ERR_INVALID_ARG, "ibf_build_batch: a plan twice");
  const int nt = std::max(1, std::min(count, nthreads > 0 ? std::min(nthreads, 64) : 8));
  // the caller's earlier work (inputs, predictor parameters) first
  {
    const hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return fail(IBF_ERR_DEVICE, std::string("ibf_build_batch: ") + hipGetErrorString(e));
    const hipError_t e2 = hipStreamSynchronize((hipStream_t)stream);
    if (e2 != hipSuccess) return fail(IBF_ERR_DEVICE, std::string("ibf_build_batch: ") + hipGetErrorString(e2));
  }
  std::atomic<int> next{0};
  std::atomic<bool> stop{false};
  std::mutex mu;
  int err_rc = IBF_OK, err_at = -1;
  std::string err_msg;
  auto worker = [&]() {
    hipStream_t st = nullptr;
    if (hipSetDevice(dev) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      std::lock_guard<std::mutex> g(mu);
      if (err_rc == IBF_OK) {
        err_rc = IBF_ERR_DEVICE;
        err_msg = "ibf_build_batch: cannot create a worker stream";
      }
      stop = true;
      return;
    }
    while (!stop) {
      const int i = next.fetch_add(1);
      if (i >= count) break;
      const int rc = ibf_build(plans[i], st);
      if (rc != IBF_OK) {
        std::lock_guard<std::mutex> g(mu);
        if (err_rc == IBF_OK || i < err_at) {
          err_rc = rc;
          err_at = i;
          err_msg = g_last_error;
        }
        stop = true;
      }
    }
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  };
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  if (err_rc != IBF_OK) {
    if (failed) *failed = err_at;
    return fail(err_rc, err_msg);
  }
  return IBF_OK;
}

int ibf_apply(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
              int64_t nrhs, void* stream) {
  if (!p) return fail(IBF_ERR_INVALID_ARG, "ibf_apply: null plan");
  if (!p->built) return fail(IBF_ERR_NOT_BUILT, "ibf_apply: plan not built");
  if (!g || !u) return fail(IBF_ERR_INVALID_ARG, "ibf_apply: null vector");
  if (nrhs < 1) return fail(IBF_ERR_INVALID_ARG, "ibf_apply: nrhs < 1");
  if (ldg < p->nxi || ldu < p->nx) return fail(IBF_ERR_INVALID_ARG, "ibf_apply: leading dimension too small");
  if (p->dim == 2) return ibf::apply2d(p, g, ldg, u, ldu, nrhs, (hipStream_t)stream);
  return ibf::apply_plan(p, g, ldg, u, ldu, nrhs, (hipStream_t)stream);
}

int ibf_apply_adjoint(ibf_plan_t p, const void* h, int64_t ldh, void* v, int64_t ldv,
                      int64_t nrhs, void* stream) {
  if (!p) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_adjoint: null plan");
  if (!p->built) return fail(IBF_ERR_NOT_BUILT, "ibf_apply_adjoint: plan not built");
  if (!h || !v) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_adjoint: null vector");
  if (nrhs < 1) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_adjoint: nrhs < 1");
  if (ldh < p->nx || ldv < p->nxi)
    return fail(IBF_ERR_INVALID_ARG, "ibf_apply_adjoint: leading dimension too small");
  if (p->dim != 1) return fail(IBF_ERR_UNSUPPORTED, "ibf_apply_adjoint: provided for dim 1");
  return ibf::apply_adjoint(p, h, ldh, v, ldv, nrhs, (hipStream_t)stream);
}

int ibf_apply_profile(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
                      int64_t nrhs, void* stream, ibf_profile* prof) {
  if (!prof) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_profile: null profile");
  if (!p) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_profile: null plan");
  if (!p->built) return fail(IBF_ERR_NOT_BUILT, "ibf_apply_profile: plan not built");
  if (!g || !u) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_profile: null vector");
  if (nrhs < 1) return fail(IBF_ERR_INVALID_ARG, "ibf_apply_profile: nrhs < 1");
  if (ldg < p->nxi || ldu < p->nx)
    return fail(IBF_ERR_INVALID_ARG, "ibf_apply_profile: leading dimension too small");
  std::memset(prof, 0, sizeof(*prof));
  if (p->dim == 2)
    return fail(IBF_ERR_UNSUPPORTED, "ibf_apply_profile: per-launch profile is for dim 1");
  return ibf::apply_plan(p, g, ldg, u, ldu, nrhs, (hipStream_t)stream, prof);
}

int ibf_query(ibf_plan_t p, ibf_info* info) {
  if (!p || !info) return fail(IBF_ERR_INVALID_ARG, "ibf_query: null argument");
  std::memset(info, 0, sizeof(*info));
  if (p->dim == 2) {
    ibf::query2d(p, info);
    return IBF_OK;
  }
  info->L = p->geo.L;
  info->l0 = p->geo.l0;
  info->h = p->geo.h;
  info->n_levels = p->geo.L - 2 * p->geo.l0 + 1;
  for (size_t i = 0; i < p->rank.size() && i < 64; ++i) info->rank[i] = p->rank[i];
  info->n_pairs = p->npairs;
  info->nnz_prelim = p->nnz_prelim;
  info->nnz_opt = p->nnz_opt;
  info->nnz_stored = p->nnz_stored;
  int64_t fb = (int64_t)(p->vbar_bytes + p->ubar_bytes + p->mdot_bytes);
  for (auto& st : p->stages) fb += (int64_t)(st.bytes + st.qbytes);
  info->factor_bytes = fb;
  info->build_ms = p->build_ms;
  info->smax_x = p->smax_x;
  info->smax_xi = p->smax_xi;
  // built: whether the sweep-in ran; before: whether it will (sweep_in = -1 resolved)
  info->sweep_in = p->built ? (p->rank_in_g.empty() ? 0 : 1) : p->sweep_in;
  for (size_t i = 0; i < p->rank_in_g.size() && i < 64; ++i) info->rank_in_g[i] = p->rank_in_g[i];
  for (size_t i = 0; i < p->rank_in_h.size() && i < 64; ++i) info->rank_in_h[i] = p->rank_in_h[i];
  info->r = p->r;
  info->tol = p->tol;
  info->learned = p->learned ? 1 : 0;
  return IBF_OK;
}

int ibf_set_allocator(ibf_alloc_fn alloc, ibf_free_fn free_fn) {
  if (!alloc != !free_fn) {
    ibf::set_error("ibf_set_allocator: give both functions or neither");
    return IBF_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = free_fn;
  return IBF_OK;
}

int ibf_destroy(ibf_plan_t p) {
  if (!p) return IBF_OK;
  if (p->dim == 2) {
    ibf::destroy2d(p);
    delete p;
    return IBF_OK;
  }
  if (!p->d_xs && !p->built) {   // never touched the device
    delete p;
    return IBF_OK;
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  ibf::free_factors(p);
  void* bufs[] = {p->d_xs, p->d_xis, p->d_perm_x, p->d_perm_xi,
                  p->d_xoff, p->d_xioff, p->d_xleaf, p->d_xileaf};
  for (void* b : bufs)
    if (b) (void)ibf::dev_free(b);
  (void)hipSetDevice(cur);
  delete p;
  return IBF_OK;
}

// Phase descriptor of the probe entry points (missing parameters take the defaults).
static int probe_phase(const char* who, int phase_id, const double* params, int n_params,
                       ibf::PhaseDesc* ph) {
  if (n_params < 0 || n_params > ibf::kMaxParams || (n_params > 0 && !params))
    return fail(IBF_ERR_INVALID_ARG, std::string(who) + ": bad phase parameters");
  const double defaults[4][3] = {{1, 0, 0}, {2, 1, 8}, {2, 1, 16}, {3, 0.3125, 0}};
  if (phase_id < 0 || phase_id > 3 || phase_id == IBF_PHASE_FIO2D)
    return fail(IBF_ERR_UNSUPPORTED, std::string(who) + ": unsupported phase");
  *ph = ibf::PhaseDesc{};
  ph->kind = phase_id;
  for (int i = 0; i < 3; ++i) ph->p[i] = i < n_params ? params[i] : defaults[phase_id][i];
  return IBF_OK;
}

int ibf_eval_kernel(int phase_id, const double* params, int n_params,
                    const double* x, const double* xi, int64_t n, void* out,
                    void* stream) {
  if (!x || !xi || !out || n < 0)
    return fail(IBF_ERR_INVALID_ARG, "ibf_eval_kernel: bad argument");
  ibf::PhaseDesc ph{};
  const int rc = probe_phase("ibf_eval_kernel", phase_id, params, n_params, &ph);
  if (rc) return rc;
  if (n == 0) return IBF_OK;
  return ibf::eval_kernel(ph, x, xi, n, out, (hipStream_t)stream);
}

int ibf_rel_error(const void* u, int64_t ldu, const void* ref, int64_t ldr, int64_t n,
                  int64_t nrhs, int precision, double* out, void* stream) {
  if (!u || !ref || !out || n < 0 || nrhs < 1 || nrhs > 65535 || ldu < n || ldr < n ||
      precision < IBF_FP64 || precision > IBF_BF16X2)
    return fail(IBF_ERR_INVALID_ARG, "ibf_rel_error: bad argument");
  return ibf::rel_error(u, ldu, ref, ldr, n, nrhs, precision, out, (hipStream_t)stream);
}

int ibf_dense_apply(int phase_id, const double* params, int n_params, const double* x,
                    int64_t n_x, const double* xi, int64_t n_xi, const void* g, int64_t ldg,
                    void* u, int64_t ldu, int64_t nrhs, void* stream) {
  if (!x || !xi || !g || !u || n_x < 0 || n_xi < 0 || nrhs < 1 || nrhs > 65535 || ldg < n_xi ||
      ldu < n_x)
    return fail(IBF_ERR_INVALID_ARG, "ibf_dense_apply: bad argument");
  ibf::PhaseDesc ph{};
  const int rc = probe_phase("ibf_dense_apply", phase_id, params, n_params, &ph);
  if (rc) return rc;
  if (n_x == 0) return IBF_OK;
  return ibf::dense_apply(ph, x, n_x, xi, n_xi, g, ldg, u, ldu, nrhs, (hipStream_t)stream);
}

int ibf_dense_apply_2d(int phase_id, const double* params, int n_params, const double* x,
                       int64_t n_x, const double* xi, int64_t n_xi, const void* g, int64_t ldg,
                       void* u, int64_t ldu, int64_t nrhs, void* stream) {
  if (!x || !xi || !g || !u || n_x < 0 || n_xi < 0 || nrhs < 1 || nrhs > 65535 || ldg < n_xi ||
      ldu < n_x)
    return fail(IBF_ERR_INVALID_ARG, "ibf_dense_apply_2d: bad argument");
  if (n_params < 0 || n_params > ibf::kMaxParams || (n_params > 0 && !params))
    return fail(IBF_ERR_INVALID_ARG, "ibf_dense_apply_2d: bad phase parameters");
  // the 2-D phases and defaults of ibf_plan with dim = 2
  const double defaults[4][3] = {{1, 0, 0}, {0, 0, 0}, {2, 1, 16}, {3, 0.3125, 0}};
  if (phase_id < 0 || phase_id > 3 || phase_id == IBF_PHASE_FIO1D)
    return fail(IBF_ERR_UNSUPPORTED, "ibf_dense_apply_2d: unsupported phase");
  ibf::PhaseDesc ph{};
  ph.kind = phase_id;
  for (int i = 0; i < 3; ++i) ph.p[i] = i < n_params ? params[i] : defaults[phase_id][i];
  if (phase_id == IBF_PHASE_FIO2D && ph.p[2] == 0.0)
    return fail(IBF_ERR_INVALID_ARG, "ibf_dense_apply_2d: p2 == 0");
  if (n_x == 0) return IBF_OK;
  return ibf::dense_apply_2d(ph, x, n_x, xi, n_xi, g, ldg, u, ldu, nrhs, (hipStream_t)stream);
}

}  // extern "C"
