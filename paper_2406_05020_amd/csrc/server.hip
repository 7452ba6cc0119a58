// Continuous-batching request server.
//
// Requests (whole IBVPs plus an evaluation grid) queue on the host.  A pool of
// worker threads, each owning one HIP stream, takes work in arrival order as
// soon as a slot is free and the estimated HBM footprint fits within the
// budget left by the work in flight.  Work is a batch: the oldest queued
// request together with the later queued requests that share its operator
// (the same grid, kernel, PDE and point layout -- only the point data differ,
// as for serving requests of one grid size), up to max_batch.  A batch is
// assembled once and solved as one multi-problem IterGP (gpfvm::batch_solve:
// every iteration applies the shared operator to all its problems in one set
// of grouped launches), then each request's posterior is evaluated on its
// own grid.  A batch of one runs the single-request path.  Batches in flight
// overlap on the device; memory comes from a shared caching allocator (no
// hipMalloc / hipFree in steady state).  Every kernel of the path is
// deterministic (fixed reduction order, no atomics in arithmetic); a request
// solved in a batch agrees with the same request solved alone to rounding
// (the batched operator takes the GEMM form of the point-block solves).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "common.h"
#include "internal.h"

using namespace gpfvm;

// PDE terms a request's memory estimate allows for (plan intermediates per term)
constexpr int EST_TERMS = 8;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Deep copy of an IBVP so that the caller may free its arrays after submit.
struct IBVPCopy {
  gpfvm_ibvp p{};
  std::vector<double> edges[3], cell_coef, f_int, coef;
  std::vector<int> alpha, cellwise;
  std::vector<gpfvm_pointgroup> groups;
  std::vector<std::array<std::vector<double>, 3>> gaxis;
  std::vector<std::vector<double>> gy;

  explicit IBVPCopy(const gpfvm_ibvp& s) {
    p = s;
    long long N = 1;
    for (int i = 0; i < s.dim; ++i) {
      edges[i].assign(s.edges[i], s.edges[i] + s.ncell[i] + 1);
      p.edges[i] = edges[i].data();
      N *= s.ncell[i];
    }
    alpha.assign(s.alpha, s.alpha + s.nterm * s.dim);
    coef.assign(s.coef, s.coef + s.nterm);
    p.alpha = alpha.data();
    p.coef = coef.data();
    if (s.cellwise) { cellwise.assign(s.cellwise, s.cellwise + s.nterm); p.cellwise = cellwise.data(); }
    bool any_cw = false;
    for (int t = 0; t < s.nterm; ++t) any_cw |= (s.cellwise && s.cellwise[t]);
    if (any_cw && s.cell_coef) { cell_coef.assign(s.cell_coef, s.cell_coef + N); p.cell_coef = cell_coef.data(); }
    else p.cell_coef = nullptr;
    if (s.f_int) { f_int.assign(s.f_int, s.f_int + N); p.f_int = f_int.data(); }
    groups.assign(s.groups, s.groups + s.ngroup);
    gaxis.resize(s.ngroup);
    gy.resize(s.ngroup);
    for (int g = 0; g < s.ngroup; ++g) {
      long long sz = 1;
      for (int i = 0; i < s.dim; ++i) {
        gaxis[g][i].assign(s.groups[g].axis[i], s.groups[g].axis[i] + s.groups[g].n[i]);
        groups[g].axis[i] = gaxis[g][i].data();
        sz *= s.groups[g].n[i];
      }
      gy[g].assign(s.groups[g].y, s.groups[g].y + sz);
      groups[g].y = gy[g].data();
    }
    p.groups = groups.data();
  }
};

}  // namespace

// Everything of an IBVP that defines its operator (all but the point data),
// as bytes: requests with equal keys share the operator and can be batched.
static std::string operator_key(const gpfvm_ibvp& p) {
  std::string k;
  auto put = [&](const void* a, size_t n) { k.append((const char*)a, n); };
  long long N = 1;
  put(&p.dim, sizeof(int));
  for (int i = 0; i < p.dim; ++i) {
    put(&p.ncell[i], sizeof(int));
    put(p.edges[i], (p.ncell[i] + 1) * sizeof(double));
    put(&p.lengthscale[i], sizeof(double));
    put(&p.kernel[i], sizeof(int));
    N *= p.ncell[i];
  }
  put(&p.outputscale, sizeof(double));
  put(&p.nterm, sizeof(int));
  put(p.alpha, (size_t)p.nterm * p.dim * sizeof(int));
  put(p.coef, p.nterm * sizeof(double));
  bool any_cw = false;
  for (int t = 0; t < p.nterm; ++t) {
    const int cw = p.cellwise ? p.cellwise[t] : 0;
    put(&cw, sizeof(int));
    any_cw |= cw != 0;
  }
  if (any_cw) put(p.cell_coef, N * sizeof(double));
  const int has_f = p.f_int ? 1 : 0;
  put(&has_f, sizeof(int));
  if (p.f_int) put(p.f_int, N * sizeof(double));
  put(&p.noise_pde, sizeof(double));
  put(&p.noise_pde_relative, sizeof(int));
  put(&p.ngroup, sizeof(int));
  for (int g = 0; g < p.ngroup; ++g) {
    const gpfvm_pointgroup& G = p.groups[g];
    for (int i = 0; i < p.dim; ++i) {
      put(&G.n[i], sizeof(int));
      put(G.axis[i], G.n[i] * sizeof(double));
      put(&G.deriv[i], sizeof(int));
    }
    put(&G.noise_var, sizeof(double));
  }
  return k;
}

struct gpfvm_request {
  long long ticket = 0;
  std::unique_ptr<IBVPCopy> ibvp;
  std::string opkey;                // operator_key of the IBVP
  std::vector<double> yobs;         // [y_b; int_V f] in observation order
  int batch = 1;                    // requests solved together with this one
  int gdim = 0;
  int gn[3] = {1, 1, 1};
  std::vector<double> gaxis[3];
  long long M = 0;
  size_t est_bytes = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  int rc = GPFVM_OK;
  bool done = false;
  std::string err;
  gpfvm_solve_info info{};
  std::vector<double> mean, var;
};

struct gpfvm_server {
  gpfvm_server_opts opts{};
  DeviceCache cache;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<gpfvm_request*> queue;
  std::map<long long, std::unique_ptr<gpfvm_request>> all;
  size_t reserved = 0;
  size_t peak_reserved = 0;
  int in_flight = 0, peak_in_flight = 0;
  long long next_ticket = 1;
  long long completed = 0;
  bool stop = false;
  int device = 0;
};

// Coarsening factors of the coarse warm start: among the nested schemes whose
// per-dimension factors divide the cell counts, the one with the most coarse
// cells that is at most `target` and coarser than the fine scheme (ties: the
// smaller largest factor).  Returns the number of coarse cells, 0 for none.
static long long choose_coarsen(const gpfvm_ibvp& p, long long target, int f[3]) {
  f[0] = f[1] = f[2] = 1;
  if (target < 1) return 0;
  std::vector<int> div[3];
  for (int i = 0; i < p.dim; ++i)
    for (int k = 1; k <= p.ncell[i]; ++k)
      if (p.ncell[i] % k == 0) div[i].push_back(k);
  for (int i = p.dim; i < 3; ++i) div[i].push_back(1);
  long long best = 0;
  int best_max = 1 << 30;
  for (int a : div[0])
    for (int b : div[1])
      for (int c : div[2]) {
        if (a == 1 && b == 1 && c == 1) continue;
        long long nc = (long long)(p.ncell[0] / a);
        if (p.dim > 1) nc *= p.ncell[1] / b;
        if (p.dim > 2) nc *= p.ncell[2] / c;
        const int mx = std::max(a, std::max(b, c));
        if (nc <= target && (nc > best || (nc == best && mx < best_max))) {
          best = nc;
          best_max = mx;
          f[0] = a; f[1] = b; f[2] = c;
        }
      }
  if (best == 0) f[0] = f[1] = f[2] = 1;
  return best;
}

// Conservative device-memory estimate of one request (bytes); n_coarse: coarse cells of the warm start.
static size_t estimate_bytes(const gpfvm_ibvp& p, int max_iter, long long M, int prec, long long n_coarse) {
  long long N = 1;
  for (int i = 0; i < p.dim; ++i) N *= p.ncell[i];
  long long nb = 0;
  for (int g = 0; g < p.ngroup; ++g) {
    long long s = 1;
    for (int i = 0; i < p.dim; ++i) s *= p.groups[g].n[i];
    nb += s;
  }
  const double d8 = 8.0;
  double b = 0;
  b += 2.0 * N * max_iter * d8;                            // directions and S D
  b += (48.0 + 6.0 * EST_TERMS) * N * d8;           // solver vectors, plan intermediates, full-Gram buffers
  b += 4.0 * nb * nb * d8;             // L, L^{-1} (and transposes)
  b += 1.0 * nb * nb * d8;             // float32 L^{-1} and L^{-T} of the row-streaming solves
  if (qform_ok(N, nb)) b += 3.0 * nb * N * d8;             // point correction Q and its build buffers
  b += 2.0 * nb * 64 * d8 + 4.0 * (nb + 64) * 64 * d8;     // Cholesky workspace
  b += 0.5 * nb * nb * d8;                                 // the triangular inverse's two workspaces
  const double chunk = (double)posterior_chunk(nb, M);
  b += (4.0 * nb + 64.0) * chunk * d8;                     // posterior point-block chunks (or the grouped form's
                                                           // factors, mode-product intermediates and solved
                                                           // columns) and column partials
  {                                                        // posterior direction batches
    const double widest = std::max(std::max((double)M, (double)N), std::max(1.0, (double)nb));
    const double B = (double)posterior_dir_batch(max_iter, (i64)widest);
    b += (2.0 * M * B + N * B + 4.0 * nb * B) * d8 + 8.0 * M * d8;
  }
  if (prec == GPFVM_PREC_MIXED) b += 12.0 * N * 4.0;       // float32 operator buffers
  if (n_coarse > 0) {                                      // C, S C^T, R, C S C^T, L^{-1} (directions: max_iter)
    b += 3.0 * n_coarse * N * d8 + 3.0 * n_coarse * n_coarse * d8;
    b += 6.0 * 64.0 * N * d8;                              // the 64-rhs operator buffers
  }
  return (size_t)(1.25 * b) + (size_t)(32 << 20);
}

// Device bytes one more problem adds to a batch: its directions and S D, its
// solver vectors and the wider multi-rhs operator buffers.
static size_t batch_extra_bytes(const gpfvm_ibvp& p, int max_iter) {
  long long N = 1, nb = 0;
  for (int i = 0; i < p.dim; ++i) N *= p.ncell[i];
  for (int g = 0; g < p.ngroup; ++g) {
    long long s = 1;
    for (int i = 0; i < p.dim; ++i) s *= p.groups[g].n[i];
    nb += s;
  }
  const double b = (2.0 * max_iter + 24.0 + 2.0 * EST_TERMS) * N * 8.0 + 8.0 * nb * 8.0 + 8.0 * max_iter;
  return (size_t)(1.25 * b);
}

int gpfvm_assemble_cached(const gpfvm_ibvp* p, const gpfvm_assemble_opts* opts, void* stream, DeviceCache* cache,
                          gpfvm_handle** out);

static void run_request(gpfvm_server* S, gpfvm_request* r, hipStream_t st) {
  gpfvm_handle* h = nullptr;
  int f[3];
  const long long n_coarse = choose_coarsen(r->ibvp->p, S->opts.coarse_cells, f);
  gpfvm_assemble_opts ao;
  gpfvm_default_assemble_opts(&ao);
  ao.max_iter = S->opts.max_iter + (int)n_coarse;
  int rc = gpfvm_assemble_cached(&r->ibvp->p, &ao, st, &S->cache, &h);
  if (rc) {
    r->rc = rc;
    r->err = gpfvm_last_error(nullptr);
    return;
  }
  gpfvm_solve_opts so;
  gpfvm_default_solve_opts(&so);
  so.prec = S->opts.prec;
  so.tol = S->opts.tol;
  so.max_iter = S->opts.max_iter;
  so.check_every = S->opts.check_every;
  if (n_coarse > 0)
    for (int i = 0; i < 3; ++i) so.coarsen[i] = f[i];
  rc = gpfvm_solve(h, &so, &r->info, st);
  if (rc && rc != GPFVM_E_NOCONV) {
    r->rc = rc;
    r->err = gpfvm_last_error(h);
    gpfvm_destroy(h);
    return;
  }
  Arena out;
  out.cache = &S->cache;
  double* dmean = (double*)out.alloc((size_t)r->M * sizeof(double));
  double* dvar = (double*)out.alloc((size_t)r->M * sizeof(double));
  if (!dmean || !dvar) {
    r->rc = GPFVM_E_NOMEM;
    r->err = "out of device memory (posterior output)";
  } else {
    const double* ax[3] = {r->gaxis[0].data(), r->gaxis[1].data(), r->gaxis[2].data()};
    rc = gpfvm_posterior(h, r->gdim, r->gn, ax, dmean, dvar, st);
    if (rc) {
      r->rc = rc;
      r->err = gpfvm_last_error(h);
    } else {
      r->mean.resize(r->M);
      r->var.resize(r->M);
      hipError_t e = hipMemcpyAsync(r->mean.data(), dmean, r->M * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(r->var.data(), dvar, r->M * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) { r->rc = GPFVM_E_HIP; r->err = hipGetErrorString(e); }
      else r->rc = r->info.status;
    }
  }
  (void)hipStreamSynchronize(st);
  out.release();
  gpfvm_destroy(h);
}

// A batch of requests sharing one operator: one assembly, one batched solve,
// a posterior per request.
static void run_batch(gpfvm_server* S, std::vector<gpfvm_request*>& rs, hipStream_t st) {
  const int R = (int)rs.size();
  for (auto* r : rs) r->batch = R;
  gpfvm_handle* h = nullptr;
  gpfvm_assemble_opts ao;
  gpfvm_default_assemble_opts(&ao);
  ao.max_iter = S->opts.max_iter;
  int rc = gpfvm_assemble_cached(&rs[0]->ibvp->p, &ao, st, &S->cache, &h);
  auto fail_all = [&](int code, const std::string& m) {
    for (auto* r : rs) { r->rc = code; r->err = m; }
  };
  if (rc) { fail_all(rc, gpfvm_last_error(nullptr)); return; }
  const long long n = (long long)rs[0]->yobs.size();
  std::vector<double> yall((size_t)R * n);
  for (int z = 0; z < R; ++z) std::memcpy(yall.data() + (size_t)z * n, rs[z]->yobs.data(), n * sizeof(double));
  std::vector<BatchResult> res;
  rc = batch_solve(h, R, yall.data(), S->opts.tol, S->opts.max_iter, S->opts.check_every, 25, st, res);
  if (rc) {
    fail_all(rc, gpfvm_last_error(h));
    gpfvm_destroy(h);
    return;
  }
  Arena out;
  out.cache = &S->cache;
  for (int z = 0; z < R; ++z) {
    gpfvm_request* r = rs[z];
    r->info.iters = res[z].iters;
    r->info.outer = 0;
    r->info.rel_res = res[z].rel_res;
    r->info.rel_res_full = std::nan("");          // not evaluated for batched requests
    r->info.coarse = 0;
    r->info.status = res[z].state == 2 ? GPFVM_E_NOTPD
                     : (S->opts.tol > 0 && res[z].rel_res > S->opts.tol) ? GPFVM_E_NOCONV : GPFVM_OK;
    double* dmean = (double*)out.alloc((size_t)r->M * sizeof(double));
    double* dvar = (double*)out.alloc((size_t)r->M * sizeof(double));
    if (!dmean || !dvar) { r->rc = GPFVM_E_NOMEM; r->err = "out of device memory (posterior output)"; continue; }
    const double* ax[3] = {r->gaxis[0].data(), r->gaxis[1].data(), r->gaxis[2].data()};
    rc = batch_posterior(h, z, r->gdim, r->gn, ax, dmean, dvar, st);
    if (rc) { r->rc = rc; r->err = gpfvm_last_error(h); continue; }
    r->mean.resize(r->M);
    r->var.resize(r->M);
    hipError_t e = hipMemcpyAsync(r->mean.data(), dmean, r->M * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(r->var.data(), dvar, r->M * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { r->rc = GPFVM_E_HIP; r->err = hipGetErrorString(e); }
    else r->rc = r->info.status == GPFVM_E_NOTPD ? GPFVM_E_NOTPD : r->info.status;
    {                                  // this request's result is ready: release it now
      std::lock_guard<std::mutex> lk(S->mu);
      r->t_done = now_s();
      r->done = true;
      S->completed += 1;
    }
    S->cv.notify_all();
  }
  (void)hipStreamSynchronize(st);
  out.release();
  gpfvm_destroy(h);
}

static void worker_main(gpfvm_server* S, int w) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[w];
  std::vector<gpfvm_request*> batch;
  size_t batch_bytes = 0;
  for (;;) {
    gpfvm_request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        if (S->stop) return true;
        if (S->queue.empty()) return false;
        return S->queue.front()->est_bytes + S->reserved <= (size_t)S->opts.hbm_budget || S->in_flight == 0;
      });
      if (S->stop && S->queue.empty()) return;
      if (S->queue.empty()) continue;
      r = S->queue.front();
      S->queue.pop_front();
      batch.assign(1, r);
      batch_bytes = r->est_bytes;
      // later queued requests with the same operator join, in arrival order, while the batch
      // stays within max_batch and the budget (float64 IterGP without the coarse start only)
      if (S->opts.max_batch > 1 && S->opts.prec == GPFVM_PREC_FP64 && S->opts.coarse_cells == 0 &&
          r->est_bytes <= (size_t)S->opts.hbm_budget) {
        const size_t extra = batch_extra_bytes(r->ibvp->p, S->opts.max_iter);
        for (auto it = S->queue.begin(); it != S->queue.end() && (int)batch.size() < S->opts.max_batch;) {
          if ((*it)->opkey == r->opkey && S->reserved + batch_bytes + extra <= (size_t)S->opts.hbm_budget) {
            batch.push_back(*it);
            batch_bytes += extra;
            it = S->queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      S->reserved += batch_bytes;
      S->peak_reserved = std::max(S->peak_reserved, S->reserved);
      S->in_flight += (int)batch.size();
      S->peak_in_flight = std::max(S->peak_in_flight, S->in_flight);
    }
    const double t0 = now_s();
    for (auto* q : batch) q->t_start = t0;
    if (r->est_bytes > (size_t)S->opts.hbm_budget) {
      r->rc = GPFVM_E_NOMEM;
      r->err = "request exceeds the server's HBM budget";
    } else {
      try {
        if (batch.size() == 1) run_request(S, r, st);
        else run_batch(S, batch, st);
      } catch (const std::exception& e) {
        for (auto* q : batch) {
          q->rc = GPFVM_E_NOMEM;
          q->err = std::string("internal error: ") + e.what();
        }
      }
    }
    const double t1 = now_s();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->reserved -= batch_bytes;
      S->in_flight -= (int)batch.size();
      for (auto* q : batch) {
        if (q->done) continue;         // released by run_batch as its posterior finished
        q->t_done = t1;
        q->done = true;
        S->completed += 1;
      }
    }
    S->cv.notify_all();
  }
}

extern "C" void gpfvm_default_server_opts(gpfvm_server_opts* o) {
  if (!o) return;
  o->workers = 8;
  o->hbm_budget = 64LL << 30;
  o->prec = GPFVM_PREC_FP64;
  o->tol = 1e-6;
  o->max_iter = 1024;
  o->check_every = 16;
  o->coarse_cells = 0;
  o->max_batch = 16;
}

extern "C" int gpfvm_server_create(const gpfvm_server_opts* o, gpfvm_server** out) {
  if (!out) return GPFVM_E_INVALID;
  *out = nullptr;
  gpfvm_server_opts def;
  gpfvm_default_server_opts(&def);
  if (!o) o = &def;
  if (o->workers < 1 || o->workers > 16 || o->hbm_budget < (1LL << 26) || o->max_iter < 1 || !(o->tol >= 0) ||
      o->check_every < 1 || (o->prec != GPFVM_PREC_FP64 && o->prec != GPFVM_PREC_MIXED) || o->coarse_cells < 0 ||
      o->coarse_cells > GPFVM_MAX_COARSE || (o->coarse_cells > 0 && o->prec != GPFVM_PREC_FP64) ||
      o->max_batch < 1 || o->max_batch > GPFVM_MAX_SERVER_BATCH)
    return GPFVM_E_INVALID;
  auto S = std::make_unique<gpfvm_server>();
  S->opts = *o;
  if (hipGetDevice(&S->device) != hipSuccess) return GPFVM_E_HIP;
  for (int w = 0; w < o->workers; ++w) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : S->streams) (void)hipStreamDestroy(x);
      return GPFVM_E_HIP;
    }
    S->streams.push_back(st);
  }
  gpfvm_server* raw = S.release();
  for (int w = 0; w < o->workers; ++w) raw->workers.emplace_back(worker_main, raw, w);
  *out = raw;
  return GPFVM_OK;
}

extern "C" int gpfvm_server_submit(gpfvm_server* S, const gpfvm_ibvp* p, int dim, const int* n,
                                   const double* const* axis, long long* ticket) {
  if (!S || !ticket) return GPFVM_E_INVALID;
  int rc = gpfvm_validate(p);
  if (rc) return rc;
  if (dim != p->dim || !n || !axis) return GPFVM_E_INVALID;
  // requests are single-output problems (the copy below keeps no system fields)
  if (p->nout > 1 || p->neq > 1 || p->term_out || p->term_eq || p->out_scale) return GPFVM_E_INVALID;
  for (int g = 0; g < p->ngroup; ++g)
    if (p->groups[g].nterm != 0 || p->groups[g].output != 0) return GPFVM_E_INVALID;
  auto r = std::make_unique<gpfvm_request>();
  r->gdim = dim;
  r->M = 1;
  for (int i = 0; i < dim; ++i) {
    if (n[i] < 1 || !axis[i]) return GPFVM_E_INVALID;
    r->gn[i] = n[i];
    r->gaxis[i].assign(axis[i], axis[i] + n[i]);
    r->M *= n[i];
  }
  r->ibvp = std::make_unique<IBVPCopy>(*p);
  r->opkey = operator_key(r->ibvp->p);
  {
    const gpfvm_ibvp& q = r->ibvp->p;
    long long N = 1;
    for (int i = 0; i < q.dim; ++i) N *= q.ncell[i];
    for (int g = 0; g < q.ngroup; ++g) {
      long long sz = 1;
      for (int i = 0; i < q.dim; ++i) sz *= q.groups[g].n[i];
      r->yobs.insert(r->yobs.end(), q.groups[g].y, q.groups[g].y + sz);
    }
    if (q.f_int) r->yobs.insert(r->yobs.end(), q.f_int, q.f_int + N);
    else r->yobs.insert(r->yobs.end(), (size_t)N, 0.0);
  }
  {
    int f[3];
    const long long n_coarse = choose_coarsen(r->ibvp->p, S->opts.coarse_cells, f);
    r->est_bytes = estimate_bytes(*p, S->opts.max_iter + (int)n_coarse, r->M, S->opts.prec, n_coarse);
  }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return GPFVM_E_STATE;
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->all[r->ticket] = std::move(r);
  }
  S->cv.notify_all();
  return GPFVM_OK;
}

extern "C" int gpfvm_server_poll(gpfvm_server* S, long long ticket, int wait, int* done, gpfvm_request_result* res,
                                 double* mean, double* var) {
  if (!S || !done) return GPFVM_E_INVALID;
  gpfvm_request* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return GPFVM_E_INVALID;
    r = it->second.get();
    if (wait) S->cv.wait(lk, [&] { return r->done; });
    *done = r->done ? 1 : 0;
  }
  if (!*done) return GPFVM_OK;
  if (res) {
    res->rc = r->rc;
    res->info = r->info;
    res->t_submit = r->t_submit;
    res->t_start = r->t_start;
    res->t_done = r->t_done;
    res->est_bytes = (long long)r->est_bytes;
    res->n_grid = r->M;
    res->batch = r->batch;
  }
  if (r->rc == GPFVM_OK || r->rc == GPFVM_E_NOCONV) {
    if (mean) std::memcpy(mean, r->mean.data(), r->M * sizeof(double));
    if (var) std::memcpy(var, r->var.data(), r->M * sizeof(double));
  }
  return GPFVM_OK;
}

extern "C" int gpfvm_server_stats(gpfvm_server* S, gpfvm_server_info* st) {
  if (!S || !st) return GPFVM_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  st->queued = (long long)S->queue.size();
  st->in_flight = S->in_flight;
  st->completed = S->completed;
  st->peak_in_flight = S->peak_in_flight;
  st->reserved_bytes = (long long)S->reserved;
  st->peak_reserved_bytes = (long long)S->peak_reserved;
  st->cached_bytes = S->cache.cached_bytes;
  st->device_bytes = S->cache.total_bytes;
  return GPFVM_OK;
}

extern "C" void gpfvm_server_destroy(gpfvm_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto st : S->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  S->cache.release_all();
  delete S;
}
