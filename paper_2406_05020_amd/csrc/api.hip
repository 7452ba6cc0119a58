// C-ABI entry points: validation, assembly of an IBVP handle, the full-Gram
// matvec, dense Gram blocks and the stand-alone factor call.
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "common.h"
#include "internal.h"

using namespace gpfvm;

static thread_local std::string g_last_error = "";

#define HIPCHK(h, expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      (h)->err = std::string("HIP error: ") + hipGetErrorString(e_) +     \
                 " at " #expr;                                            \
      return GPFVM_E_HIP;                                                 \
    }                                                                     \
  } while (0)

static int fail_static(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

extern "C" void gpfvm_default_assemble_opts(gpfvm_assemble_opts* o) {
  if (!o) return;
  o->max_iter = 512;
  o->tile = GPFVM_TILE_FP32;
  o->reuse_memory = 1;
}

namespace {
// Per-device block caches of standalone handles (reuse_memory).
std::mutex g_cache_mu;
std::map<int, std::unique_ptr<DeviceCache>> g_caches;

DeviceCache* process_cache() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto& c = g_caches[dev];
  if (!c) c = std::make_unique<DeviceCache>();
  return c.get();
}
}  // namespace

extern "C" long long gpfvm_release_cached_memory(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  long long freed = 0;
  for (auto& kv : g_caches) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    freed += (long long)kv.second->trim();
  }
  (void)hipSetDevice(cur);
  return freed;
}

extern "C" void gpfvm_default_solve_opts(gpfvm_solve_opts* o) {
  if (!o) return;
  o->prec = GPFVM_PREC_FP64;
  o->tol = 1e-8;
  o->max_iter = 512;
  o->resume = 0;
  o->tile = GPFVM_TILE_FP32;
  o->block = 32;
  o->max_outer = 1000;
  o->check_every = 8;
  o->reorth_passes = 2;
  o->replace_every = 25;
  for (int k = 0; k < GPFVM_MAX_DIM; ++k) o->coarsen[k] = 1;
  o->method = GPFVM_METHOD_ITERGP;
}

// ---------------------------------------------------------------------------
// validation (no HIP calls)
// ---------------------------------------------------------------------------
static bool finite_arr(const double* a, long long n) {
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

extern "C" int gpfvm_validate(const gpfvm_ibvp* p) {
  if (!p) return fail_static(GPFVM_E_INVALID, "ibvp is NULL");
  if (p->dim < 2 || p->dim > GPFVM_MAX_DIM) return fail_static(GPFVM_E_INVALID, "dim must be 2 or 3");
  long long N = 1;
  for (int i = 0; i < p->dim; ++i) {
    if (p->ncell[i] < 1 || p->ncell[i] > (1 << 20))
      return fail_static(GPFVM_E_INVALID, "ncell[" + std::to_string(i) + "] out of range");
    if (!p->edges[i]) return fail_static(GPFVM_E_INVALID, "edges[" + std::to_string(i) + "] is NULL");
    if (!finite_arr(p->edges[i], p->ncell[i] + 1))
      return fail_static(GPFVM_E_INVALID, "edges[" + std::to_string(i) + "] not finite");
    for (int j = 0; j < p->ncell[i]; ++j)
      if (!(p->edges[i][j + 1] > p->edges[i][j]))
        return fail_static(GPFVM_E_INVALID, "edges[" + std::to_string(i) + "] not strictly increasing");
    if (!(p->lengthscale[i] > 0) || !std::isfinite(p->lengthscale[i]))
      return fail_static(GPFVM_E_INVALID, "lengthscale must be positive");
    if (p->kernel[i] < GPFVM_KERNEL_SE || p->kernel[i] > GPFVM_KERNEL_MATERN72)
      return fail_static(GPFVM_E_INVALID, "kernel[" + std::to_string(i) + "] unknown");
    N *= p->ncell[i];
  }
  // a Matern-(q + 1/2) dimension admits derivative orders up to q
  auto order_cap = [&](int i) { return p->kernel[i] == GPFVM_KERNEL_SE ? GPFVM_MAX_DERIV : p->kernel[i] - 1; };
  if (N > (1LL << 31) - 1) return fail_static(GPFVM_E_INVALID, "too many volumes");
  if (!(p->outputscale > 0) || !std::isfinite(p->outputscale))
    return fail_static(GPFVM_E_INVALID, "outputscale must be positive");
  if (p->nout < 0 || p->nout > GPFVM_MAX_OUTPUTS) return fail_static(GPFVM_E_INVALID, "nout out of range");
  if (p->neq < 0 || p->neq > GPFVM_MAX_TERMS) return fail_static(GPFVM_E_INVALID, "neq out of range");
  const int nout = std::max(1, p->nout), neq = std::max(1, p->neq);
  if (p->out_scale)
    for (int o = 0; o < nout; ++o)
      if (!(p->out_scale[o] > 0) || !std::isfinite(p->out_scale[o]))
        return fail_static(GPFVM_E_INVALID, "out_scale must be positive");
  if (p->nterm < 1 || p->nterm > GPFVM_MAX_TERMS) return fail_static(GPFVM_E_INVALID, "nterm out of range");
  if (!p->alpha || !p->coef) return fail_static(GPFVM_E_INVALID, "alpha/coef is NULL");
  bool any_cw = false;
  std::vector<int> eq_used(neq, 0), out_used(nout, 0);
  for (int t = 0; t < p->nterm; ++t) {
    const int to = p->term_out ? p->term_out[t] : 0, te = p->term_eq ? p->term_eq[t] : 0;
    if (to < 0 || to >= nout) return fail_static(GPFVM_E_INVALID, "term_out out of range");
    if (te < 0 || te >= neq) return fail_static(GPFVM_E_INVALID, "term_eq out of range");
    eq_used[te] = 1;
    out_used[to] = 1;
    for (int i = 0; i < p->dim; ++i) {
      const int a = p->alpha[t * p->dim + i];
      if (a < 0 || a > GPFVM_MAX_DERIV)
        return fail_static(GPFVM_E_INVALID, "derivative order out of range [0, 4]");
      if (a > order_cap(i))
        return fail_static(GPFVM_E_INVALID, "derivative order above the smoothness of the Matern kernel in dim " +
                                                std::to_string(i));
    }
    if (!std::isfinite(p->coef[t])) return fail_static(GPFVM_E_INVALID, "coef not finite");
    if (p->cellwise && p->cellwise[t]) any_cw = true;
  }
  for (int e = 0; e < neq; ++e)
    if (!eq_used[e]) return fail_static(GPFVM_E_INVALID, "equation " + std::to_string(e) + " has no term");
  if (any_cw) {
    if (!p->cell_coef) return fail_static(GPFVM_E_INVALID, "cellwise term without cell_coef");
    if (!finite_arr(p->cell_coef, N)) return fail_static(GPFVM_E_INVALID, "cell_coef not finite");
  }
  if ((long long)neq * N > (1LL << 31) - 1) return fail_static(GPFVM_E_INVALID, "too many volume observations");
  if (p->f_int && !finite_arr(p->f_int, (long long)neq * N)) return fail_static(GPFVM_E_INVALID, "f_int not finite");
  if (!(p->noise_pde > 0) || !std::isfinite(p->noise_pde))
    return fail_static(GPFVM_E_INVALID, "noise_pde must be positive");
  if (p->ngroup < 0 || p->ngroup > GPFVM_MAX_GROUPS) return fail_static(GPFVM_E_INVALID, "ngroup out of range");
  if (p->ngroup > 0 && !p->groups) return fail_static(GPFVM_E_INVALID, "groups is NULL");
  long long nb = 0;
  for (int g = 0; g < p->ngroup; ++g) {
    const gpfvm_pointgroup& G = p->groups[g];
    long long sz = 1;
    for (int i = 0; i < p->dim; ++i) {
      if (G.n[i] < 1) return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": n < 1");
      if (!G.axis[i]) return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": axis NULL");
      if (!finite_arr(G.axis[i], G.n[i])) return fail_static(GPFVM_E_INVALID, "group axis not finite");
      if (G.deriv[i] < 0 || G.deriv[i] > GPFVM_MAX_DERIV)
        return fail_static(GPFVM_E_INVALID, "group derivative order out of range [0, 4]");
      if (G.deriv[i] > order_cap(i))
        return fail_static(GPFVM_E_INVALID, "group derivative order above the smoothness of the Matern kernel in dim " +
                                                std::to_string(i));
      sz *= G.n[i];
    }
    if (G.nterm < 0 || G.nterm > GPFVM_MAX_PTERMS)
      return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": nterm out of range");
    if (G.nterm == 0) {
      if (G.output < 0 || G.output >= nout)
        return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": output out of range");
      if (!out_used[G.output])
        return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": its output appears in no equation");
    } else {
      if (!G.terms) return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": terms is NULL");
      for (int c = 0; c < G.nterm; ++c) {
        const gpfvm_pointterm& T = G.terms[c];
        if (T.output < 0 || T.output >= nout || !out_used[T.output])
          return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": a term's output is out of range or "
                                              "appears in no equation");
        if (!std::isfinite(T.coef)) return fail_static(GPFVM_E_INVALID, "group term coef not finite");
        for (int i = 0; i < p->dim; ++i) {
          if (T.deriv[i] < 0 || T.deriv[i] > GPFVM_MAX_DERIV || T.deriv[i] > order_cap(i))
            return fail_static(GPFVM_E_INVALID, "group term derivative order out of range in dim " + std::to_string(i));
          if (T.weight[i] && !finite_arr(T.weight[i], G.n[i]))
            return fail_static(GPFVM_E_INVALID, "group term weight not finite");
        }
      }
    }
    if (!G.y) return fail_static(GPFVM_E_INVALID, "group " + std::to_string(g) + ": y is NULL");
    if (!finite_arr(G.y, sz)) return fail_static(GPFVM_E_INVALID, "group y not finite");
    if (!(G.noise_var > 0) || !std::isfinite(G.noise_var))
      return fail_static(GPFVM_E_INVALID, "group noise_var must be positive");
    nb += sz;
  }
  if (nb > 65536) return fail_static(GPFVM_E_INVALID, "more than 65536 point observations");
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
static int upload(gpfvm_handle* h, const double* src, size_t n, double** dst) {
  *dst = (double*)h->arena.alloc(std::max<size_t>(n, 1) * sizeof(double));
  if (!*dst) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
  if (n) HIPCHK(h, hipMemcpyAsync(*dst, src, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return GPFVM_OK;
}

// Factor matrix of dimension `dim` (its lengthscale and kernel).
static int make_factor(gpfvm_handle* h, int kind, int p, int q, int n1, const double* a1, int n2,
                       const double* a2, int dim, Factor& f) {
  f.n1 = n1;
  f.n2 = n2;
  f.d = (double*)h->arena.alloc((size_t)n1 * n2 * sizeof(double));
  if (!f.d) { h->err = "out of device memory (factor)"; return GPFVM_E_NOMEM; }
  HIPCHK(h, launch_factor(kind, h->kq[dim], p, q, n1, a1, n2, a2, h->ell[dim], 1.0, f.d, n2, h->stream));
  return GPFVM_OK;
}

static int add_f32_copy(gpfvm_handle* h, Factor& f) {
  if (f.f) return GPFVM_OK;
  f.f = (float*)h->arena.alloc((size_t)f.n1 * f.n2 * sizeof(float));
  if (!f.f) { h->err = "out of device memory (factor f32)"; return GPFVM_E_NOMEM; }
  HIPCHK(h, launch_copy_f64_to_f32(f.d, f.f, (i64)f.n1 * f.n2, h->stream));
  return GPFVM_OK;
}

static void merge_terms(gpfvm_handle* h) {
  // (L_V k L_V')  =  sum_{a, a'} c_a c_a' prod_i F^{a_i a'_i}, F^{pq} = (-1)^q D(p+q)
  // (Sec. 3.2 eq. LkL): merge pairs with the same orders, scaling flags and equation
  // block.  Only terms on the same output pair up (k = diag(s_i k), Sec. 3.3), and each
  // merged coefficient carries that output's outputscale.
  h->gterms.clear();
  for (auto& t1 : h->pterms)
    for (auto& t2 : h->pterms) {
      if (t1.out != t2.out) continue;
      GramTerm g;
      int asum = 0;
      for (int i = 0; i < h->d; ++i) {
        g.m[i] = t1.alpha[i] + t2.alpha[i];
        asum += t2.alpha[i];
      }
      g.coef = h->sfo[t1.out] * t1.coef * t2.coef * ((asum & 1) ? -1.0 : 1.0);
      g.lflag = t1.cellwise;
      g.rflag = t2.cellwise;
      g.e1 = t1.eq;
      g.e2 = t2.eq;
      bool merged = false;
      for (auto& e : h->gterms)
        if (e.lflag == g.lflag && e.rflag == g.rflag && e.e1 == g.e1 && e.e2 == g.e2 && e.m[0] == g.m[0] &&
            e.m[1] == g.m[1] && e.m[2] == g.m[2]) {
          e.coef += g.coef;
          merged = true;
          break;
        }
      if (!merged) h->gterms.push_back(g);
    }
  h->gterms.erase(std::remove_if(h->gterms.begin(), h->gterms.end(), [](const GramTerm& g) { return g.coef == 0.0; }),
                  h->gterms.end());
}

static int build_ops(gpfvm_handle* h) {
  const int d = h->d;
  const i64 Nc = h->Nc;
  // ---- volume block: one operator per equation (its block row of the volume Gram) ----
  h->op_pp.assign(h->neq, KronOp());
  for (int e = 0; e < h->neq; ++e) {
    KronOp& op = h->op_pp[e];
    op.d = d;
    for (int i = 0; i < d; ++i) op.in_shape[i] = op.out_shape[i] = h->nc[i];
    op.in_len = h->N;
    op.out_off = (i64)e * Nc;
  }
  if (d == 2) {
    // pre-sum the last-dimension matrices of terms sharing (m_0, L, R, block)
    struct Key { int m0, l, r, e1, e2; };
    std::vector<Key> keys;
    std::vector<std::vector<const GramTerm*>> members;
    for (auto& g : h->gterms) {
      size_t k = 0;
      for (; k < keys.size(); ++k)
        if (keys[k].m0 == g.m[0] && keys[k].l == g.lflag && keys[k].r == g.rflag && keys[k].e1 == g.e1 &&
            keys[k].e2 == g.e2)
          break;
      if (k == keys.size()) { keys.push_back({g.m[0], g.lflag, g.rflag, g.e1, g.e2}); members.emplace_back(); }
      members[k].push_back(&g);
    }
    h->combos.clear();
    h->combos.reserve(keys.size());
    for (size_t k = 0; k < keys.size(); ++k) {
      Factor c;
      c.n1 = c.n2 = h->nc[1];
      c.d = (double*)h->arena.alloc((size_t)c.n1 * c.n2 * sizeof(double));
      if (!c.d) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
      std::vector<const double*> mats;
      std::vector<double> cf;
      for (auto* g : members[k]) { mats.push_back(h->Dfac[{1, g->m[1]}].d); cf.push_back(g->coef); }
      for (size_t s0 = 0; s0 < mats.size(); s0 += 8) {
        // (at most 8 per pass; accumulate by chaining with the partial result)
        std::vector<const double*> mm(mats.begin() + s0, mats.begin() + std::min(mats.size(), s0 + 8));
        std::vector<double> cc(cf.begin() + s0, cf.begin() + std::min(cf.size(), s0 + 8));
        if (s0 > 0) { mm.push_back(c.d); cc.push_back(1.0); }
        HIPCHK(h, launch_lincomb((int)mm.size(), mm.data(), cc.data(), (i64)c.n1 * c.n2, c.d, h->stream));
      }
      h->combos.push_back(c);
      KronTerm t{};
      t.M[0] = h->Dfac[{0, keys[k].m0}].d; t.ld[0] = h->nc[0];
      t.M[1] = h->combos.back().d; t.ld[1] = h->nc[1];
      t.alpha = 1.0;
      t.lscale = keys[k].l; t.rscale = keys[k].r;
      t.in_off = (i64)keys[k].e2 * Nc;
      h->op_pp[keys[k].e1].terms.push_back(t);
    }
  } else {
    for (auto& g : h->gterms) {
      KronTerm t{};
      for (int i = 0; i < d; ++i) { t.M[i] = h->Dfac[{i, g.m[i]}].d; t.ld[i] = h->nc[i]; }
      t.alpha = g.coef;
      t.lscale = g.lflag; t.rscale = g.rflag;
      t.in_off = (i64)g.e2 * Nc;
      h->op_pp[g.e1].terms.push_back(t);
    }
  }
  for (int e = 0; e < h->neq; ++e)
    if (h->op_pp[e].terms.empty()) {
      h->err = "the volume Gram's block row of equation " + std::to_string(e) + " is identically zero";
      return GPFVM_E_INVALID;
    }
  // ---- cross blocks: per point group, every (point component, PDE term) pair on one output ----
  h->op_bp.clear();
  h->op_pb.clear();
  const size_t T = h->pterms.size();
  for (size_t gi = 0; gi < h->groups.size(); ++gi) {
    const Group& G = h->groups[gi];
    KronOp bp;
    bp.d = d;
    for (int i = 0; i < d; ++i) { bp.in_shape[i] = h->nc[i]; bp.out_shape[i] = G.n[i]; }
    bp.in_len = h->N; bp.out_off = G.offset;
    std::vector<KronOp> pb(h->neq);
    for (int e = 0; e < h->neq; ++e) {
      pb[e].d = d;
      for (int i = 0; i < d; ++i) { pb[e].in_shape[i] = G.n[i]; pb[e].out_shape[i] = h->nc[i]; }
      pb[e].in_len = h->nb;
      pb[e].out_off = (i64)e * Nc;
    }
    for (size_t c = 0; c < G.comps.size(); ++c)
      for (size_t ti = 0; ti < T; ++ti) {
        const PdeTerm& P = h->pterms[ti];
        if (P.out != G.comps[c].out) continue;
        KronTerm a{}, b{};
        for (int i = 0; i < d; ++i) {
          a.M[i] = b.M[i] = h->Qfac[gi][c * T + ti][i].d;
          a.ld[i] = b.ld[i] = h->nc[i];
          b.trans[i] = 1;
        }
        a.alpha = b.alpha = h->sfo[P.out] * G.comps[c].coef * P.coef;
        a.rscale = P.cellwise;
        a.in_off = (i64)P.eq * Nc;
        b.lscale = P.cellwise;
        b.in_off = G.offset;
        bp.terms.push_back(a);
        pb[P.eq].terms.push_back(b);
      }
    if (bp.terms.empty()) { h->err = "a point group shares no output with the equations"; return GPFVM_E_INVALID; }
    h->op_bp.push_back(bp);
    for (auto& o : pb)
      if (!o.terms.empty()) h->op_pb.push_back(o);
  }
  return GPFVM_OK;
}

// float32 operators: same structure on float32 copies of the factors
int gpfvm::build_ops32(gpfvm_handle* h) {
  for (auto& kv : h->Dfac) { int rc = add_f32_copy(h, kv.second); if (rc) return rc; }
  for (auto& c : h->combos) { int rc = add_f32_copy(h, c); if (rc) return rc; }
  for (auto& g : h->Qfac)
    for (auto& t : g)
      for (int i = 0; i < h->d; ++i) { int rc = add_f32_copy(h, t[i]); if (rc) return rc; }
  auto to32 = [&](const void* p) -> const void* {
    for (auto& kv : h->Dfac) if (kv.second.d == p) return kv.second.f;
    for (auto& c : h->combos) if (c.d == p) return c.f;
    for (auto& g : h->Qfac) for (auto& t : g) for (int i = 0; i < h->d; ++i) if (t[i].d == p) return t[i].f;
    return nullptr;
  };
  auto conv = [&](const KronOp& a) {
    KronOp b = a;
    for (auto& t : b.terms)
      for (int i = 0; i < h->d; ++i) t.M[i] = to32(t.M[i]);
    return b;
  };
  h->op_pp32.clear();
  for (auto& o : h->op_pp) h->op_pp32.push_back(conv(o));
  h->op_bp32.clear(); h->op_pb32.clear();
  for (auto& o : h->op_bp) h->op_bp32.push_back(conv(o));
  for (auto& o : h->op_pb) h->op_pb32.push_back(conv(o));
  if (h->cellc && !h->cellc_f) {
    h->cellc_f = (float*)h->arena.alloc((size_t)h->N * sizeof(float));
    if (!h->cellc_f) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
    HIPCHK(h, launch_copy_f64_to_f32(h->cellc, h->cellc_f, h->N, h->stream));
  }
  if (h->nb > 0 && !h->Linv_f) {
    h->Linv_f = (float*)h->arena.alloc((size_t)h->nb * h->nb * sizeof(float));
    if (!h->Linv_f) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
    HIPCHK(h, launch_copy_f64_to_f32(h->Linv, h->Linv_f, (i64)h->nb * h->nb, h->stream));
  }
  return GPFVM_OK;
}


// rows (columns) of a row-major n1 x n2 factor times per-point weights wr (wc); null: 1
__global__ void k_scale_rows_cols(double* __restrict__ A, int n1, int n2, const double* __restrict__ wr,
                                  const double* __restrict__ wc) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (i64)n1 * n2) return;
  double v = A[i];
  if (wr) v *= wr[i / n2];
  if (wc) v *= wc[i % n2];
  A[i] = v;
}

hipError_t gpfvm::scale_rows_cols(double* A, int n1, int n2, const double* wr, const double* wc, hipStream_t s) {
  if (!wr && !wc) return hipSuccess;
  const i64 n = (i64)n1 * n2;
  hipLaunchKernelGGL(k_scale_rows_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, n1, n2, wr, wc);
  return hipGetLastError();
}

static int assemble_impl(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, hipStream_t s, gpfvm_handle* h) {
  const int d = p->dim;
  h->d = d;
  h->stream = s;
  h->Nc = 1;
  for (int i = 0; i < d; ++i) {
    h->nc[i] = p->ncell[i];
    h->Nc *= p->ncell[i];
    h->ell[i] = p->lengthscale[i];
    h->kq[i] = p->kernel[i] == GPFVM_KERNEL_SE ? -1 : p->kernel[i] - 1;
    h->edges_h[i].assign(p->edges[i], p->edges[i] + p->ncell[i] + 1);
  }
  h->nout = std::max(1, p->nout);
  h->neq = std::max(1, p->neq);
  h->N = h->Nc * h->neq;
  for (int o = 0; o < h->nout; ++o) h->sfo[o] = p->out_scale ? p->out_scale[o] : p->outputscale;
  h->sf2 = h->sfo[0];
  h->multi = h->nout > 1 || h->neq > 1;
  h->max_iter = opts ? std::max(1, opts->max_iter) : 512;
  h->tile = opts ? opts->tile : GPFVM_TILE_FP32;
  for (int t = 0; t < p->nterm; ++t) {
    PdeTerm P;
    for (int i = 0; i < d; ++i) P.alpha[i] = p->alpha[t * d + i];
    P.coef = p->coef[t];
    P.cellwise = (p->cellwise && p->cellwise[t]) ? 1 : 0;
    P.out = p->term_out ? p->term_out[t] : 0;
    P.eq = p->term_eq ? p->term_eq[t] : 0;
    h->pterms.push_back(P);
  }
  h->has_cc = 0;
  for (auto& P : h->pterms) h->has_cc |= P.cellwise;
  i64 off = 0;
  for (int g = 0; g < p->ngroup; ++g) {
    Group G;
    const gpfvm_pointgroup& S = p->groups[g];
    G.size = 1;
    for (int i = 0; i < d; ++i) {
      G.n[i] = S.n[i];
      G.axis[i].assign(S.axis[i], S.axis[i] + S.n[i]);
      G.size *= S.n[i];
    }
    if (S.nterm == 0) {
      PointComp c;
      for (int i = 0; i < d; ++i) c.deriv[i] = S.deriv[i];
      c.out = S.output;
      G.comps.push_back(c);
    } else {
      h->multi = true;
      for (int k = 0; k < S.nterm; ++k) {
        PointComp c;
        for (int i = 0; i < d; ++i) {
          c.deriv[i] = S.terms[k].deriv[i];
          if (S.terms[k].weight[i]) c.w[i].assign(S.terms[k].weight[i], S.terms[k].weight[i] + S.n[i]);
        }
        c.coef = S.terms[k].coef;
        c.out = S.terms[k].output;
        G.comps.push_back(c);
      }
    }
    for (int i = 0; i < d; ++i) G.deriv[i] = G.comps[0].deriv[i];
    G.noise = S.noise_var;
    G.offset = off;
    off += G.size;
    h->groups.push_back(G);
  }
  h->nb = (int)off;
  h->n = h->nb + h->N;
  merge_terms(h);
  if (h->gterms.empty()) { h->err = "the operator's volume Gram is identically zero"; return GPFVM_E_INVALID; }

  // ---- inputs to HBM ----
  int rc;
  for (int i = 0; i < d; ++i)
    if ((rc = upload(h, h->edges_h[i].data(), h->edges_h[i].size(), &h->edges[i]))) return rc;
  if (h->has_cc) {
    // the per-cell coefficient once per equation block, so every block of the volume vector
    // finds its cell's value at the same offset
    std::vector<double> cc((size_t)h->N);
    for (int e = 0; e < h->neq; ++e) std::memcpy(&cc[(size_t)e * h->Nc], p->cell_coef, (size_t)h->Nc * sizeof(double));
    if ((rc = upload(h, cc.data(), cc.size(), &h->cellc))) return rc;
  }
  {
    std::vector<double> y((size_t)h->n, 0.0);
    for (int g = 0; g < p->ngroup; ++g)
      std::memcpy(&y[h->groups[g].offset], p->groups[g].y, h->groups[g].size * sizeof(double));
    if (p->f_int) std::memcpy(&y[h->nb], p->f_int, (size_t)h->N * sizeof(double));
    if ((rc = upload(h, y.data(), y.size(), &h->yobs))) return rc;
  }

  // ---- 1-D factors (closed form) ----
  for (auto& g : h->gterms)
    for (int i = 0; i < d; ++i) {
      auto key = std::make_pair(i, g.m[i]);
      if (h->Dfac.count(key)) continue;
      Factor f;
      if ((rc = make_factor(h, 0, g.m[i], 0, h->nc[i], h->edges[i], h->nc[i], h->edges[i], i, f))) return rc;
      h->Dfac[key] = f;
    }
  std::vector<std::array<double*, 3>> gaxis(h->groups.size());
  // per-point weights of the point components on the device: [group][comp][dim] (null: 1)
  std::vector<std::vector<std::array<double*, 3>>> gw(h->groups.size());
  for (size_t g = 0; g < h->groups.size(); ++g) {
    for (int i = 0; i < d; ++i)
      if ((rc = upload(h, h->groups[g].axis[i].data(), h->groups[g].axis[i].size(), &gaxis[g][i]))) return rc;
    gw[g].resize(h->groups[g].comps.size());
    for (size_t c = 0; c < h->groups[g].comps.size(); ++c)
      for (int i = 0; i < 3; ++i) {
        gw[g][c][i] = nullptr;
        const auto& w = h->groups[g].comps[c].w[i];
        if (i < d && !w.empty())
          if ((rc = upload(h, w.data(), w.size(), &gw[g][c][i]))) return rc;
      }
  }
  const size_t T = h->pterms.size();
  h->Qfac.assign(h->groups.size(), std::vector<std::array<Factor, 3>>());
  for (size_t g = 0; g < h->groups.size(); ++g) {
    const Group& G = h->groups[g];
    h->Qfac[g].resize(G.comps.size() * T);
    for (size_t c = 0; c < G.comps.size(); ++c)
      for (size_t t = 0; t < T; ++t) {
        if (h->pterms[t].out != G.comps[c].out) continue;
        for (int i = 0; i < d; ++i) {
          Factor& f = h->Qfac[g][c * T + t][i];
          if ((rc = make_factor(h, 1, G.comps[c].deriv[i], h->pterms[t].alpha[i], G.n[i], gaxis[g][i], h->nc[i],
                                h->edges[i], i, f)))
            return rc;
          HIPCHK(h, scale_rows_cols(f.d, f.n1, f.n2, gw[g][c][i], nullptr, s));
        }
      }
  }
  GramMeta* Mp = new (std::nothrow) GramMeta;
  if (!Mp) { h->err = "host allocation failed"; return GPFVM_E_NOMEM; }
  std::unique_ptr<GramMeta> Mown(Mp);
  GramMeta& M = *Mp;
  std::memset(&M, 0, sizeof(M));
  for (size_t g1 = 0; g1 < h->groups.size(); ++g1)
    for (size_t g2 = 0; g2 < h->groups.size(); ++g2) {
      const Group &A = h->groups[g1], &B = h->groups[g2];
      for (size_t c1 = 0; c1 < A.comps.size(); ++c1)
        for (size_t c2 = 0; c2 < B.comps.size(); ++c2) {
          if (A.comps[c1].out != B.comps[c2].out) continue;
          M.pcoef[g1][c1][g2][c2] = h->sfo[A.comps[c1].out] * A.comps[c1].coef * B.comps[c2].coef;
          for (int i = 0; i < d; ++i) {
            Factor f;
            if ((rc = make_factor(h, 2, A.comps[c1].deriv[i], B.comps[c2].deriv[i], A.n[i], gaxis[g1][i], B.n[i],
                                  gaxis[g2][i], i, f)))
              return rc;
            HIPCHK(h, scale_rows_cols(f.d, f.n1, f.n2, gw[g1][c1][i], gw[g2][c2][i], s));
            M.Pp[g1][c1][g2][c2][i] = f.d;
          }
        }
    }

  // ---- PDE noise ----
  if (p->noise_pde_relative) {
    // mean over the volume observations of diag(L_V k L_V'): for equation e the merged
    // terms of block (e, e), sum_terms coef L R prod_i D_i(m_i)[j_i, j_i] (coef with s_out)
    std::map<std::pair<int, int>, std::vector<double>> diag;
    for (auto& kv : h->Dfac) {
      const int n1 = kv.second.n1;
      std::vector<double> full((size_t)n1 * n1);
      HIPCHK(h, hipMemcpyAsync(full.data(), kv.second.d, full.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
      std::vector<double> dg(n1);
      for (int j = 0; j < n1; ++j) dg[j] = full[(size_t)j * n1 + j];
      diag[kv.first] = dg;
    }
    std::vector<std::array<const double*, 3>> dp(h->gterms.size());
    for (size_t t = 0; t < h->gterms.size(); ++t)
      for (int i = 0; i < d; ++i) dp[t][i] = diag[{i, h->gterms[t].m[i]}].data();
    double acc = 0;
    int idx[3];
    for (i64 v = 0; v < h->Nc; ++v) {
      i64 r = v;
      for (int i = d - 1; i >= 0; --i) { idx[i] = (int)(r % h->nc[i]); r /= h->nc[i]; }
      double sv = 0;
      for (size_t t = 0; t < h->gterms.size(); ++t) {
        const GramTerm& g = h->gterms[t];
        if (g.e1 != g.e2) continue;
        double w = g.coef;
        if (g.lflag) w *= p->cell_coef[v];
        if (g.rflag) w *= p->cell_coef[v];
        for (int i = 0; i < d; ++i) w *= dp[t][i][idx[i]];
        sv += w;
      }
      acc += sv;
    }
    h->sig_pde = p->noise_pde * acc / (double)h->N;
  } else {
    h->sig_pde = p->noise_pde;
  }

  // ---- dense-entry metadata (point block, dense Gram tiles) ----
  M.d = d; M.nb = h->nb; M.ngroup = (int)h->groups.size(); M.nterm = (int)T;
  M.ngterm = (int)h->gterms.size();
  M.neq = h->neq;
  M.Nc = h->Nc;
  if (M.ngterm > MAXGT) { h->err = "too many merged operator terms"; return GPFVM_E_INVALID; }
  for (int i = 0; i < d; ++i) M.nc[i] = h->nc[i];
  for (int i = d; i < 3; ++i) M.nc[i] = 1;
  for (size_t g = 0; g < h->groups.size(); ++g) {
    const Group& G = h->groups[g];
    for (int i = 0; i < 3; ++i) M.gn[g][i] = (i < d) ? G.n[i] : 1;
    M.goff[g] = G.offset;
    M.gnoise[g] = G.noise;
    M.gcomp[g] = (int)G.comps.size();
    for (size_t c = 0; c < G.comps.size(); ++c)
      for (size_t t = 0; t < T; ++t) {
        if (h->pterms[t].out != G.comps[c].out) continue;
        M.qcoef[g][c][t] = h->sfo[G.comps[c].out] * G.comps[c].coef * h->pterms[t].coef;
        for (int i = 0; i < d; ++i) M.Qp[g][c][t][i] = h->Qfac[g][c * T + t][i].d;
      }
  }
  M.goff[h->groups.size()] = h->nb;
  for (size_t t = 0; t < T; ++t) { M.tcw[t] = h->pterms[t].cellwise; M.teq[t] = h->pterms[t].eq; }
  for (size_t t = 0; t < h->gterms.size(); ++t) {
    for (int i = 0; i < 3; ++i) M.gm[t][i] = h->gterms[t].m[i];
    M.gcoef[t] = h->gterms[t].coef; M.gl[t] = h->gterms[t].lflag; M.gr[t] = h->gterms[t].rflag;
    M.ge1[t] = h->gterms[t].e1; M.ge2[t] = h->gterms[t].e2;
  }
  for (auto& kv : h->Dfac) M.Dp[kv.first.first][kv.first.second] = kv.second.d;
  M.cellc = h->cellc;
  M.sig_pde = h->sig_pde;
  h->meta = (GramMeta*)h->arena.alloc(sizeof(GramMeta));
  if (!h->meta) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
  HIPCHK(h, hipMemcpyAsync(h->meta, &M, sizeof(M), hipMemcpyHostToDevice, s));

  // ---- point block: G_bb, Cholesky, inverse factor ----
  if (h->nb > 0) {
    h->L = (double*)h->arena.alloc((size_t)h->nb * h->nb * sizeof(double));
    h->Linv = (double*)h->arena.alloc((size_t)h->nb * h->nb * sizeof(double));
    if (!h->L || !h->Linv) { h->err = "out of device memory (point block)"; return GPFVM_E_NOMEM; }
    HIPCHK(h, launch_gram_block(h->meta, 0, h->nb, 0, h->nb, h->L, h->nb, s));
    rc = cholesky_and_inverse(h->L, h->Linv, h->nb, h->arena, s, h->err);
    if (rc) return rc;
    {   // transposed copies: every triangular product then streams rows
      h->Lt = (double*)h->arena.alloc((size_t)h->nb * h->nb * sizeof(double));
      h->Linvt = (double*)h->arena.alloc((size_t)h->nb * h->nb * sizeof(double));
      if (!h->Lt || !h->Linvt) { h->err = "out of device memory (point block)"; return GPFVM_E_NOMEM; }
      HIPCHK(h, launch_transpose(h->L, h->Lt, h->nb, s));
      HIPCHK(h, launch_transpose(h->Linv, h->Linvt, h->nb, s));
    }
  }
  if ((rc = build_ops(h))) return rc;
  HIPCHK(h, hipStreamSynchronize(s));
  return GPFVM_OK;
}

// Host-side checks of the assemble arguments (no HIP call).
static int check_assemble_args(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, gpfvm_handle** out) {
  if (!out) return fail_static(GPFVM_E_INVALID, "out is NULL");
  *out = nullptr;
  int rc = gpfvm_validate(p);
  if (rc) return rc;
  if (opts && (opts->max_iter < 1 || opts->max_iter > (1 << 20)))
    return fail_static(GPFVM_E_INVALID, "max_iter out of range");
  if (opts && opts->tile != GPFVM_TILE_FP32 && opts->tile != GPFVM_TILE_BF16X3)
    return fail_static(GPFVM_E_INVALID, "tile: GPFVM_TILE_FP32 or GPFVM_TILE_BF16X3");
  return GPFVM_OK;
}

int gpfvm_assemble_cached(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, void* stream, DeviceCache* cache,
                          gpfvm_handle** out);

extern "C" int gpfvm_assemble(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, void* stream,
                              gpfvm_handle** out) {
  int rc = check_assemble_args(p, opts, out);
  if (rc) return rc;
  const bool reuse = !opts || opts->reuse_memory != 0;
  DeviceCache* cache = reuse ? process_cache() : nullptr;
  rc = gpfvm_assemble_cached(p, opts, stream, cache, out);
  if (rc == GPFVM_OK && out && *out) (*out)->process_cache = (cache != nullptr);
  return rc;
}

int gpfvm_assemble_cached(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, void* stream, DeviceCache* cache,
                          gpfvm_handle** out) {
  int rc = check_assemble_args(p, opts, out);
  if (rc) return rc;
  gpfvm_handle* h = new (std::nothrow) gpfvm_handle();
  if (!h) return fail_static(GPFVM_E_NOMEM, "host allocation failed");
  h->arena.cache = cache;
  try {
    rc = assemble_impl(p, opts, (hipStream_t)stream, h);
  } catch (const std::exception& e) {
    h->err = std::string("internal error: ") + e.what();
    rc = GPFVM_E_NOMEM;
  }
  if (rc) {
    g_last_error = h->err;
    (void)hipStreamSynchronize((hipStream_t)stream);
    h->arena.release();
    delete h;
    return rc;
  }
  *out = h;
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// full-Gram matvec
// ---------------------------------------------------------------------------

int gpfvm::get_full_ops(gpfvm_handle* h, int nrhs, gpfvm_opset** out) {
  auto it = h->full_ops.find(nrhs);
  if (it != h->full_ops.end()) { *out = it->second.get(); return GPFVM_OK; }
  auto os = std::make_unique<gpfvm_opset>();
  os->nrhs = nrhs;
  const i64 n = h->n, nb = h->nb;
  os->XF = (double*)h->arena.alloc((size_t)n * nrhs * sizeof(double));
  os->YF = (double*)h->arena.alloc((size_t)n * nrhs * sizeof(double));
  os->TB = (double*)h->arena.alloc((size_t)std::max<i64>(nb, 1) * nrhs * sizeof(double));
  if (!os->XF || !os->YF || !os->TB) { h->err = "out of device memory"; return GPFVM_E_NOMEM; }
  // bind with explicit strides (vectors are [points; volumes] of length n)
  int rc = compile_kron_list(h->op_pp, F64, nrhs, os->XF + nb, n, os->YF + nb, n, h->cellc, h->cellc, 0.0,
                             os->XF + nb, h->sig_pde, pp_accumulate(h), h->arena, h->stream, os->pp, h->err);
  if (rc) return rc;
  if (nb > 0) {
    rc = compile_kron_list(h->op_bp, F64, nrhs, os->XF + nb, n, os->YF, n, h->cellc, h->cellc, 0.0, nullptr, 0, 0,
                           h->arena, h->stream, os->bp, h->err);
    if (rc) return rc;
    rc = compile_kron_list(h->op_pb, F64, nrhs, os->XF, n, os->YF + nb, n, h->cellc, h->cellc, 1.0, nullptr, 0, 1,
                           h->arena, h->stream, os->pb, h->err);
    if (rc) return rc;
    // TB[r] = L^T x_b[r] ; YF_b[r] += L TB[r]
    os->gbb_t.descs.push_back(desc1(os->TB, nb, os->XF, n, 1, h->L, nb, 1, nrhs, (int)nb, (int)nb, 1.0, 0.0, 4));
    os->gbb_l.descs.push_back(desc1(os->YF, n, os->TB, nb, 1, h->L, 1, nb, nrhs, (int)nb, (int)nb, 1.0, 1.0, 3));
    std::vector<Stage> st{os->gbb_t, os->gbb_l};
    if (upload_stages(st, h->arena, h->stream) != hipSuccess) { h->err = "upload failed"; return GPFVM_E_HIP; }
    os->gbb_t = st[0];
    os->gbb_l = st[1];
  }
  *out = os.get();
  h->full_ops[nrhs] = std::move(os);
  return GPFVM_OK;
}

extern "C" int gpfvm_matvec(gpfvm_handle* h, int nrhs, const void* x, void* y, int dtype, int prec, void* stream) {
  if (!h) return fail_static(GPFVM_E_INVALID, "handle is NULL");
  if (nrhs < 1 || nrhs > 4096 || !x || !y) { h->err = "matvec: bad nrhs or NULL buffer"; return GPFVM_E_INVALID; }
  if (prec != GPFVM_PREC_FP64 && prec != GPFVM_PREC_MIXED) { h->err = "matvec: bad prec"; return GPFVM_E_INVALID; }
  if (prec == GPFVM_PREC_MIXED && h->multi) { h->err = "matvec: the mixed path takes single-output problems"; return GPFVM_E_INVALID; }
  if (dtype != GPFVM_DTYPE_F64 && dtype != GPFVM_DTYPE_F32) { h->err = "matvec: bad dtype"; return GPFVM_E_INVALID; }
  const size_t esz = dtype == GPFVM_DTYPE_F64 ? sizeof(double) : sizeof(float);
  const size_t bytes = (size_t)h->n * nrhs * esz;
  if ((const char*)x < (const char*)y + bytes && (const char*)y < (const char*)x + bytes) {
    h->err = "matvec: x and y overlap";
    return GPFVM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  gpfvm_opset* os = nullptr;
  int rc = get_full_ops(h, nrhs, &os);
  if (rc) return rc;
  const i64 nn = h->n * nrhs;
  if (dtype == GPFVM_DTYPE_F64) HIPCHK(h, hipMemcpyAsync(os->XF, x, bytes, hipMemcpyDeviceToDevice, s));
  else HIPCHK(h, launch_copy_f32_to_f64((const float*)x, os->XF, nn, s));
  if (h->nb > 0) {
    HIPCHK(h, run_plan(os->bp, s));
    HIPCHK(h, launch_gemm_stage(F64, os->gbb_t, s));
    HIPCHK(h, launch_gemm_stage(F64, os->gbb_l, s));
  }
  if (prec == GPFVM_PREC_FP64) {
    HIPCHK(h, run_plan(os->pp, s));
  } else {
    // volume block through the low-precision plan (the handle's tile format), everything else float64
    gpfvm_sop* so = nullptr;
    rc = get_sop(h, nrhs, F32, &so);
    if (rc) return rc;
    const i64 n = h->n, N = h->N, nb = h->nb;
    for (int r = 0; r < nrhs; ++r)
      HIPCHK(h, launch_copy_f64_to_f32(os->XF + r * n + nb, (float*)so->X32 + r * N, N, s));
    HIPCHK(h, run_plan(so->pp, s));
    for (int r = 0; r < nrhs; ++r)
      HIPCHK(h, launch_copy_f32_to_f64((const float*)so->Y32 + r * N, os->YF + r * n + nb, N, s));
  }
  if (h->nb > 0) HIPCHK(h, run_plan(os->pb, s));
  if (dtype == GPFVM_DTYPE_F64) HIPCHK(h, hipMemcpyAsync(y, os->YF, bytes, hipMemcpyDeviceToDevice, s));
  else HIPCHK(h, launch_copy_f64_to_f32(os->YF, (float*)y, nn, s));
  return GPFVM_OK;
}

extern "C" int gpfvm_volume_matvec(gpfvm_handle* h, int nrhs, const double* x, double* y, int prec, void* stream) {
  if (!h) return fail_static(GPFVM_E_INVALID, "handle is NULL");
  if (nrhs < 1 || nrhs > 4096 || !x || !y) { h->err = "volume_matvec: bad nrhs or NULL buffer"; return GPFVM_E_INVALID; }
  if (prec != GPFVM_PREC_FP64 && prec != GPFVM_PREC_MIXED) { h->err = "volume_matvec: bad prec"; return GPFVM_E_INVALID; }
  if (prec == GPFVM_PREC_MIXED && h->multi) { h->err = "volume_matvec: the mixed path takes single-output problems"; return GPFVM_E_INVALID; }
  const size_t bytes = (size_t)h->N * nrhs * sizeof(double);
  if ((const char*)x < (const char*)y + bytes && (const char*)y < (const char*)x + bytes) {
    h->err = "volume_matvec: x and y overlap";
    return GPFVM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  if (prec == GPFVM_PREC_MIXED) {
    gpfvm_sop* so = nullptr;
    int rc = get_sop(h, nrhs, F32, &so);
    if (rc) return rc;
    HIPCHK(h, launch_copy_f64_to_f32(x, (float*)so->X32, (i64)h->N * nrhs, s));
    HIPCHK(h, run_plan(so->pp, s));
    HIPCHK(h, launch_copy_f32_to_f64((const float*)so->Y32, y, (i64)h->N * nrhs, s));
    return GPFVM_OK;
  }
  auto key = std::make_tuple((const void*)x, (void*)y, nrhs);
  auto it = h->vplans.find(key);
  if (it == h->vplans.end()) {
    // bind the plan to the caller's buffers (registered for the plan's bounds check)
    register_range(x, bytes);
    register_range(y, bytes);
    h->user_ranges.push_back(x);
    h->user_ranges.push_back(y);
    auto pl = std::make_unique<Plan>();
    int rc = compile_kron_list(h->op_pp, F64, nrhs, x, h->N, y, h->N, h->cellc, h->cellc, 0.0, x, h->sig_pde,
                               pp_accumulate(h), h->arena, s, *pl, h->err);
    if (rc) return rc;
    it = h->vplans.emplace(key, std::move(pl)).first;
  }
  HIPCHK(h, run_plan(*it->second, s));
  return GPFVM_OK;
}

extern "C" int gpfvm_gram_block(gpfvm_handle* h, long long r0, long long nr, long long c0, long long nc, double* out,
                                long long ld, void* stream) {
  if (!h) return fail_static(GPFVM_E_INVALID, "handle is NULL");
  if (r0 < 0 || c0 < 0 || nr < 0 || nc < 0 || r0 + nr > h->n || c0 + nc > h->n || ld < nc || !out) {
    h->err = "gram_block: range out of bounds";
    return GPFVM_E_INVALID;
  }
  HIPCHK(h, launch_gram_block(h->meta, r0, nr, c0, nc, out, ld, (hipStream_t)stream));
  return GPFVM_OK;
}

extern "C" int gpfvm_factor(int kind, int kernel, int p, int q, int n1, const double* a1, int n2, const double* a2,
                            double lengthscale, double* out, void* stream) {
  if (kind < 0 || kind > 2) return fail_static(GPFVM_E_INVALID, "factor: kind must be 0, 1 or 2");
  if (kernel < GPFVM_KERNEL_SE || kernel > GPFVM_KERNEL_MATERN72) return fail_static(GPFVM_E_INVALID, "factor: unknown kernel");
  if (p < 0 || q < 0 || p + q > 2 * GPFVM_MAX_DERIV) return fail_static(GPFVM_E_INVALID, "factor: bad orders");
  const int kq = kernel == GPFVM_KERNEL_SE ? -1 : kernel - 1;
  if (kq >= 0 && (p > kq || q > kq))
    return fail_static(GPFVM_E_INVALID, "factor: order above the smoothness of the Matern kernel");
  if (n1 < 1 || n2 < 1 || !a1 || !a2 || !out) return fail_static(GPFVM_E_INVALID, "factor: bad sizes/pointers");
  if (!(lengthscale > 0)) return fail_static(GPFVM_E_INVALID, "factor: lengthscale must be positive");
  const int l1 = (kind == 0) ? n1 + 1 : n1;
  const int l2 = (kind == 2) ? n2 : n2 + 1;
  if (!finite_arr(a1, l1) || !finite_arr(a2, l2)) return fail_static(GPFVM_E_INVALID, "factor: non-finite input");
  hipStream_t s = (hipStream_t)stream;
  double *d1 = nullptr, *d2 = nullptr;
  if (hipMalloc(&d1, l1 * sizeof(double)) != hipSuccess || hipMalloc(&d2, l2 * sizeof(double)) != hipSuccess) {
    if (d1) (void)hipFree(d1);
    return fail_static(GPFVM_E_NOMEM, "factor: device allocation failed");
  }
  hipError_t e = hipMemcpyAsync(d1, a1, l1 * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d2, a2, l2 * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_factor(kind, kq, p, q, n1, d1, n2, d2, lengthscale, 1.0, out, n2, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d1);
  (void)hipFree(d2);
  if (e != hipSuccess) return fail_static(GPFVM_E_HIP, std::string("factor: ") + hipGetErrorString(e));
  return GPFVM_OK;
}

extern "C" int gpfvm_get_info(const gpfvm_handle* h, gpfvm_handle_info* info) {
  if (!h || !info) return fail_static(GPFVM_E_INVALID, "NULL argument");
  info->dim = h->d;
  info->n_pde = h->N;
  info->n_b = h->nb;
  info->n = h->n;
  info->noise_pde_var = h->sig_pde;
  info->device_bytes = h->arena.bytes;
  info->volume_launches = 0;
  for (auto& kv : h->vplans) { info->volume_launches = (int)kv.second->stages.size(); break; }
  info->volume_flops = h->vplans.empty() ? 0.0 : h->vplans.begin()->second->flops;
  return GPFVM_OK;
}

extern "C" void gpfvm_destroy(gpfvm_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  // cached blocks are handed to the next handle at once: wait for any work the
  // caller may still have queued on other streams (hipFree would as well)
  if (h->process_cache) (void)hipDeviceSynchronize();
  for (const void* p : h->user_ranges) unregister_range(p);
  h->arena.release();
  delete h;
}

extern "C" const char* gpfvm_last_error(const gpfvm_handle* h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}
