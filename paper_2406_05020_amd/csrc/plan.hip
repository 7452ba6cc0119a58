// Compiler of Kronecker-sum operators into stages of grouped MFMA GEMMs.
//
// A KronOp is y = sum_s alpha_s (L_s o) (M_{s,0} x ... x M_{s,d-1}) (R_s o x_s)
// (Sec. 3.2 eq. LkL and Sec. 4.1 eq. kronecker-structure: the operator
// distributes over the 1-D factors, so each product is a chain of 1-D mode
// products, "cheap" Kronecker matvecs).  Mode products are applied in the
// same dimension order for every term (most-contracting dimension first);
// common chain prefixes are shared; the last mode product of every term is
// summed inside one GEMM via multiple K-segments, with the per-volume scaling
// L_s applied in the epilogue (slot 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>

#include "common.h"
#include "internal.h"

namespace gpfvm {

// ---------------------------------------------------------------------------
// Registry of live device ranges.  Every GEMM descriptor is checked against it
// on the host before upload, so a plan that would address memory outside a
// buffer is reported as an error instead of reaching the GPU.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_reg_mu;
std::map<uintptr_t, size_t>& registry() {
  static std::map<uintptr_t, size_t> r;
  return r;
}
}  // namespace

void register_range(const void* p, size_t nbytes) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  registry()[(uintptr_t)p] = nbytes;
}

void unregister_range(const void* p) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  registry().erase((uintptr_t)p);
}

bool range_ok(const void* p, size_t nbytes) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto& r = registry();
  const uintptr_t a = (uintptr_t)p;
  auto it = r.upper_bound(a);
  if (it == r.begin()) return false;
  --it;
  return a >= it->first && a + nbytes <= it->first + it->second;
}

void* DeviceCache::get(size_t nbytes) {
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = free_blocks.lower_bound(nbytes);
    if (it != free_blocks.end() && it->first <= 2 * nbytes + 4096) {
      void* p = it->second;
      cached_bytes -= (i64)it->first;
      free_blocks.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, nbytes) != hipSuccess) {
    // give the cached blocks back to the runtime and try once more
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : free_blocks) {
      (void)hipFree(kv.second);
      sizes.erase(kv.second);
      total_bytes -= (i64)kv.first;
    }
    free_blocks.clear();
    cached_bytes = 0;
    if (hipMalloc(&p, nbytes) != hipSuccess) return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  sizes[p] = nbytes;
  total_bytes += (i64)nbytes;
  return p;
}

void DeviceCache::put(void* p) {
  std::lock_guard<std::mutex> lk(mu);
  auto it = sizes.find(p);
  if (it == sizes.end()) return;
  free_blocks.emplace(it->second, p);
  cached_bytes += (i64)it->second;
}

i64 DeviceCache::trim() {
  std::lock_guard<std::mutex> lk(mu);
  i64 freed = 0;
  for (auto& kv : free_blocks) {
    (void)hipFree(kv.second);
    sizes.erase(kv.second);
    freed += (i64)kv.first;
  }
  free_blocks.clear();
  total_bytes -= freed;
  cached_bytes = 0;
  return freed;
}

void DeviceCache::release_all() {
  std::lock_guard<std::mutex> lk(mu);
  for (auto& kv : free_blocks) (void)hipFree(kv.second);
  free_blocks.clear();
  sizes.clear();
  cached_bytes = total_bytes = 0;
}

void* Arena::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 256;
  nbytes = (nbytes + 255) & ~(size_t)255;
  if (fixed) {
    if (nbytes > fixed_cap - fixed_used) return nullptr;
    void* p = fixed + fixed_used;
    fixed_used += nbytes;
    regs.push_back(p);
    register_range(p, nbytes);
    return p;
  }
  auto block = [&](size_t n) -> void* {
    void* q = nullptr;
    if (cache) q = cache->get(n);
    else if (hipMalloc(&q, n) != hipSuccess) q = nullptr;
    if (q) {
      ptrs.push_back(q);
      bytes += (i64)n;
    }
    return q;
  };
  void* p = nullptr;
  if (nbytes > ARENA_SLAB / 4) {
    p = block(nbytes);
  } else {
    if (nbytes > slab_left) {
      slab = (char*)block(ARENA_SLAB);
      slab_left = slab ? ARENA_SLAB : 0;
    }
    if (slab) {
      p = slab + (ARENA_SLAB - slab_left);
      slab_left -= nbytes;
    }
  }
  if (!p) return nullptr;
  regs.push_back(p);
  register_range(p, nbytes);
  return p;
}

void Arena::release() {
  for (void* p : regs) unregister_range(p);
  regs.clear();
  fixed_used = 0;
  for (void* p : ptrs) {
    if (cache) cache->put(p);
    else (void)hipFree(p);
  }
  ptrs.clear();
  slab = nullptr;
  slab_left = 0;
  bytes = 0;
}

namespace {

struct Tensor {            // a bound operand: base pointer, per-rhs stride, shape
  const void* p;
  i64 rhs_stride;
  int shape[3];
};

i64 prod(const int* s, int a, int b) {
  i64 r = 1;
  for (int i = a; i < b; ++i) r *= s[i];
  return r;
}

// Fill segment operands for the mode product along `dim` of tensor `in`
// (shape sh) with matrix (M, ld, trans) giving rows x cols, output `out`.
// Returns descriptors (one, or one per rhs when strides do not batch).
struct ModeGeom {
  i64 P, Q;
  int rows, cols;
};

void mode_seg(Seg& S, const ModeGeom& g, const Tensor& in, const void* M, i64 ld, int trans, double alpha,
              int slot) {
  std::memset(&S, 0, sizeof(S));
  S.alpha = alpha;
  S.slot = slot;
  S.K = g.cols;
  if (g.Q == 1) {
    // C (P x rows) = X (P x cols) * Mop^T ; batches are right-hand sides
    S.A = in.p; S.a_rs = g.cols; S.a_cs = 1; S.a_bs = in.rhs_stride;
    S.B = M;
    if (!trans) { S.b_rs = 1; S.b_cs = ld; } else { S.b_rs = ld; S.b_cs = 1; }
    S.b_bs = 0;
  } else {
    // C_p (rows x Q) = Mop (rows x cols) * X_p (cols x Q) ; batches are p (x rhs)
    S.A = M;
    if (!trans) { S.a_rs = ld; S.a_cs = 1; } else { S.a_rs = 1; S.a_cs = ld; }
    S.a_bs = 0;
    S.B = in.p; S.b_rs = g.Q; S.b_cs = 1;
    S.b_bs = (g.P == 1) ? in.rhs_stride : g.cols * g.Q;
  }
}

}  // namespace

// Byte size of one element of a plan.
static size_t esize(Elt e) { return e == F64 ? sizeof(double) : sizeof(float); }

int compile_kron_list(const std::vector<KronOp>& ops, Elt elt, int nrhs, const void* x, i64 x_rhs_stride,
                      void* y, i64 y_rhs_stride, const void* scale_src, const double* escale64, double beta,
                      const void* addx, double gamma, int accumulate, Arena& arena, hipStream_t s, Plan& out,
                      std::string& err) {
  out = Plan();
  out.elt = elt;
  out.nrhs = nrhs;
  out.x = x;
  out.y = y;
  out.scale_src = scale_src;
  if (ops.empty()) { err = "empty Kronecker operator"; return GPFVM_E_INVALID; }
  const int d = ops[0].d;
  const size_t es = esize(elt);

  // scaled input (volume-shaped inputs only)
  bool need_xs = false;
  for (auto& op : ops)
    for (auto& t : op.terms) need_xs |= (t.rscale != 0);
  // Per-volume input scaling applies to volume inputs only: the whole input of
  // every rhs (in_len values: one block of prod(in_shape) volumes per equation)
  // is scaled once, and a scaled term reads its block at in_off.
  i64 xs_len = 0;
  for (auto& op : ops)
    for (auto& t : op.terms)
      if (t.rscale) {
        const i64 len = op.in_len;
        if (t.in_off + prod(op.in_shape, 0, op.d) > len || (xs_len && xs_len != len) || len > x_rhs_stride) {
          err = "internal error: per-volume scaling of a non-volume input";
          return GPFVM_E_INVALID;
        }
        xs_len = len;
      }
  if (need_xs) {
    if (!scale_src) { err = "operator needs per-volume coefficients"; return GPFVM_E_INVALID; }
    out.in_len = xs_len;
    out.xs = arena.alloc((size_t)xs_len * nrhs * es);
    if (!out.xs) { err = "out of device memory (plan)"; return GPFVM_E_NOMEM; }
    Prescale ps;
    ps.x = x; ps.coef = scale_src; ps.xs = out.xs; ps.len = xs_len; ps.x_stride = x_rhs_stride; ps.nrhs = nrhs;
    if (!range_ok(ps.x, (size_t)((nrhs - 1) * x_rhs_stride + xs_len) * es) || !range_ok(ps.coef, (size_t)xs_len * es)) {
      err = "internal error: per-volume scaling reads outside its buffers";
      return GPFVM_E_INVALID;
    }
    out.pre.push_back(ps);
  }

  std::vector<Stage> mid(d > 1 ? d - 1 : 0);
  std::vector<Stage> fin;
  double flops = 0;

  for (size_t oi = 0; oi < ops.size(); ++oi) {
    const KronOp& op = ops[oi];
    // dimension order: most contracting first (rows/cols ascending), ties: last dim first
    std::vector<int> order(d);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const double ra = (double)op.out_shape[a] / op.in_shape[a];
      const double rb = (double)op.out_shape[b] / op.in_shape[b];
      if (ra != rb) return ra < rb;
      return a > b;
    });
    // chain prefix cache: key -> tensor
    std::map<std::vector<i64>, Tensor> cache;
    struct Pending { Tensor in; const KronTerm* t; int shape[3]; };
    std::vector<Pending> finals;
    for (const KronTerm& t : op.terms) {
      Tensor cur;
      cur.p = (t.rscale ? (const char*)out.xs : (const char*)x) + (size_t)t.in_off * es;
      cur.rhs_stride = t.rscale ? xs_len : x_rhs_stride;
      for (int i = 0; i < 3; ++i) cur.shape[i] = op.in_shape[i];
      std::vector<i64> key = {t.rscale, t.in_off};
      for (int k = 0; k + 1 < d; ++k) {
        const int dim = order[k];
        key.push_back(dim);
        key.push_back((i64)(uintptr_t)t.M[dim]);
        key.push_back(t.trans[dim]);
        auto it = cache.find(key);
        if (it != cache.end()) { cur = it->second; continue; }
        ModeGeom g;
        g.P = prod(cur.shape, 0, dim);
        g.Q = prod(cur.shape, dim + 1, d);
        g.cols = cur.shape[dim];
        g.rows = op.out_shape[dim];
        Tensor nxt;
        for (int i = 0; i < 3; ++i) nxt.shape[i] = cur.shape[i];
        nxt.shape[dim] = g.rows;
        const i64 len = prod(nxt.shape, 0, d);
        nxt.rhs_stride = len;
        void* buf = arena.alloc((size_t)len * nrhs * es);
        if (!buf) { err = "out of device memory (plan intermediate)"; return GPFVM_E_NOMEM; }
        nxt.p = buf;
        const bool batch_ok = (g.Q == 1) || (g.P == 1) || (nrhs == 1) ||
                              (cur.rhs_stride == g.P * g.cols * g.Q);   // output is contiguous
        const int ndesc = batch_ok ? 1 : nrhs;
        for (int r = 0; r < ndesc; ++r) {
          GemmDesc D;
          std::memset(&D, 0, sizeof(D));
          Tensor in = cur;
          if (!batch_ok) in.p = (const char*)cur.p + (size_t)r * cur.rhs_stride * es;
          mode_seg(D.seg[0], g, in, t.M[dim], t.ld[dim], t.trans[dim], 1.0, 0);
          D.nseg = 1;
          char* cbase = (char*)buf + (batch_ok ? 0 : (size_t)r * len * es);
          D.C = cbase;
          if (g.Q == 1) {
            D.M = (int)g.P; D.N = g.rows; D.batch = batch_ok ? nrhs : 1;
            D.c_rs = g.rows; D.c_cs = 1; D.c_bs = len;
          } else {
            D.M = g.rows; D.N = (int)g.Q; D.batch = (int)(g.P * (batch_ok ? nrhs : 1));
            D.c_rs = g.Q; D.c_cs = 1; D.c_bs = (g.P == 1) ? len : (i64)g.rows * g.Q;
          }
          flops += 2.0 * D.M * D.N * (double)g.cols * D.batch;
          mid[k].descs.push_back(D);
        }
        cache[key] = nxt;
        cur = nxt;
      }
      Pending pnd;
      pnd.in = cur;
      pnd.t = &t;
      for (int i = 0; i < 3; ++i) pnd.shape[i] = cur.shape[i];
      finals.push_back(pnd);
    }
    // final summing mode product along order[d-1]
    const int dim = order[d - 1];
    ModeGeom g;
    g.P = prod(finals[0].shape, 0, dim);
    g.Q = prod(finals[0].shape, dim + 1, d);
    g.cols = finals[0].shape[dim];
    g.rows = op.out_shape[dim];
    const i64 olen = prod(op.out_shape, 0, d);
    const bool any_l = std::any_of(op.terms.begin(), op.terms.end(), [](const KronTerm& t) { return t.lscale; });
    bool batch_ok = (nrhs == 1) || (g.Q == 1) || (g.P == 1);
    if (!batch_ok) {   // P > 1, Q > 1, several rhs: one batch stride must serve (rhs, p)
      batch_ok = !any_l && y_rhs_stride == olen;
      for (auto& f : finals)
        if (f.in.rhs_stride != g.P * g.cols * g.Q) batch_ok = false;
    }
    const int nrdesc = batch_ok ? 1 : nrhs;
    for (size_t c0 = 0; c0 < finals.size(); c0 += MAXSEG) {
      const size_t c1 = std::min(finals.size(), c0 + MAXSEG);
      // disjoint outputs share one launch per chunk index; sums need one per chunk
      const size_t slot_idx = accumulate ? fin.size() : c0 / MAXSEG;
      if (slot_idx >= fin.size()) fin.resize(slot_idx + 1);
      Stage& st = fin[slot_idx];
      for (int r = 0; r < nrdesc; ++r) {
        GemmDesc D;
        std::memset(&D, 0, sizeof(D));
        D.nseg = (int)(c1 - c0);
        for (size_t j = c0; j < c1; ++j) {
          Tensor in = finals[j].in;
          if (!batch_ok) in.p = (const char*)in.p + (size_t)r * in.rhs_stride * es;
          const KronTerm& t = *finals[j].t;
          mode_seg(D.seg[j - c0], g, in, t.M[dim], t.ld[dim], t.trans[dim], t.alpha, t.lscale ? 1 : 0);
          flops += 2.0 * (double)g.P * g.rows * g.Q * g.cols * (batch_ok ? nrhs : 1);
        }
        char* cbase = (char*)y + (size_t)op.out_off * es + (batch_ok ? 0 : (size_t)r * y_rhs_stride * es);
        D.C = cbase;
        const bool first_write = (accumulate ? oi == 0 : true) && c0 == 0;
        D.beta = first_write ? beta : 1.0;
        if (g.Q == 1) {
          D.M = (int)g.P; D.N = g.rows; D.batch = batch_ok ? nrhs : 1;
          D.c_rs = g.rows; D.c_cs = 1; D.c_bs = y_rhs_stride;
          D.e_rs = g.rows; D.e_cs = 1; D.e_bs = 0;
        } else {
          D.M = g.rows; D.N = (int)g.Q; D.batch = (int)(g.P * (batch_ok ? nrhs : 1));
          D.c_rs = g.Q; D.c_cs = 1; D.c_bs = (g.P == 1) ? y_rhs_stride : (i64)g.rows * g.Q;
          D.e_rs = g.Q; D.e_cs = 1; D.e_bs = (g.P == 1) ? 0 : (i64)g.rows * g.Q;
        }
        if (any_l) {
          if (!escale64) { err = "operator needs per-volume coefficients"; return GPFVM_E_INVALID; }
          D.escale = escale64 + op.out_off;   // the coefficients of this output block
        }
        if (first_write && addx && (oi == 0 || !accumulate)) {
          D.X = (const char*)addx + (size_t)op.out_off * es + (batch_ok ? 0 : (size_t)r * y_rhs_stride * es);
          D.x_rs = D.c_rs; D.x_cs = D.c_cs; D.x_bs = D.c_bs;
          D.gamma = gamma;
        }
        st.descs.push_back(D);
      }
    }
  }
  for (auto& m : mid)
    if (!m.descs.empty()) out.stages.push_back(m);
  for (auto& f : fin) out.stages.push_back(f);
  {
    const hipError_t e = upload_stages(out.stages, arena, s, elt);
    if (e == hipErrorInvalidValue) { err = "internal error: Kronecker plan failed its bounds check"; return GPFVM_E_INVALID; }
    if (e != hipSuccess) { err = "plan upload failed"; return GPFVM_E_HIP; }
  }
  out.flops = flops;
  return GPFVM_OK;
}

int compile_kron(const KronOp& op, Elt elt, int nrhs, const void* x, void* y, const void* scale_src,
                 const double* escale64, double beta, const void* addx, double gamma, Arena& arena,
                 hipStream_t s, Plan& out, std::string& err) {
  std::vector<KronOp> ops{op};
  return compile_kron_list(ops, elt, nrhs, x, op.in_len, y, prod(op.out_shape, 0, op.d), scale_src, escale64,
                           beta, addx, gamma, 1, arena, s, out, err);
}

int merge_plans(const std::vector<const Plan*>& parts, Arena& arena, hipStream_t s, Plan& out, std::string& err) {
  out = Plan();
  if (parts.empty()) return GPFVM_OK;
  out.elt = parts[0]->elt;
  size_t nst = 0;
  for (const Plan* q : parts) {
    if (q->elt != out.elt) { err = "merge of plans with different element types"; return GPFVM_E_INVALID; }
    out.pre.insert(out.pre.end(), q->pre.begin(), q->pre.end());
    nst = std::max(nst, q->stages.size());
    out.flops += q->flops;
  }
  out.stages.resize(nst);
  for (const Plan* q : parts)
    for (size_t i = 0; i < q->stages.size(); ++i)
      out.stages[i].descs.insert(out.stages[i].descs.end(), q->stages[i].descs.begin(), q->stages[i].descs.end());
  const hipError_t e = upload_stages(out.stages, arena, s, out.elt);
  if (e == hipErrorInvalidValue) { err = "internal error: merged plan failed its bounds check"; return GPFVM_E_INVALID; }
  if (e != hipSuccess) { err = "plan upload failed"; return GPFVM_E_HIP; }
  return GPFVM_OK;
}

hipError_t run_plan(const Plan& p, hipStream_t s) {
  hipError_t e;
  for (const Prescale& ps : p.pre) {
    e = launch_scale(p.elt, ps.x, ps.x_stride, ps.coef, ps.xs, ps.len, ps.len, ps.nrhs, s);
    if (e != hipSuccess) return e;
  }
  for (const Stage& st : p.stages) {
    e = launch_gemm_stage(p.elt, st, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gpfvm
