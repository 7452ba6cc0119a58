// Solve and posterior: exact conditioning on the point observations, then
// IterGP with CG actions on the volume observations under the conditioned
// prior (Sec. 4.1 IterGP, Sec. 4.2 Cholesky preconditioner), optional mixed-
// precision iterative refinement, and the posterior mean / combined variance
// on a tensor grid (Sec. 2.1 eq. lin-cond-mean, eq. lin-cond-cov).
//
// Volume system (block elimination of G = [[G_bb, G_bp], [G_pb, G_pp + s2 I]]):
//   S = G_pp + s2 I - G_pb G_bb^{-1} G_bp,   b = y_p - G_pb G_bb^{-1} y_b.
// IterGP with CG actions, every step in float64:
//   r = b - S v ; s = r ; z = S s ; d = s - D (eta^{-1} o D^T z) ;
//   eta_i = z^T d ; v += (s^T r / eta_i) d ; store d, eta_i.
// The combined posterior uses C_i = sum_j d_j d_j^T / eta_j as S^{-1}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "common.h"
#include "internal.h"
#include "reduce.h"

using namespace gpfvm;

#define HIPCHK(h, expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      (h)->err = std::string("HIP error: ") + hipGetErrorString(e_) +     \
                 " at " #expr;                                            \
      return GPFVM_E_HIP;                                                 \
    }                                                                     \
  } while (0)

namespace {

// guarded update (two-pass form): a = (s.r)/eta with s = r;
// v += a d ; r -= a w ; X = r ; store d, w, eta ; count the iteration.
// eta comes from the previous kernel's per-workgroup partials (eta_part,
// n_eta values) or from scal[1].  s.r = r.r comes from the previous update's
// partials (rr_in, n_rr values) or from scal[0] (already tested by the dot
// kernel).  Every workgroup sums the partials itself in the same fixed order,
// so no workgroup waits on another.  With rr_in this kernel also runs the
// stopping test (converged if r.r <= tol^2 b.b: scal[4] = tol^2,
// scal[3] = b.b).  rr_out receives this update's partials of the new r.r.
//
// With vbest the kernel also guards against divergence past the attainable
// accuracy: a tolerance below it leaves the recursive residual stalled, and
// the iterations that follow lose conjugacy and grow it without bound.  The
// smallest r.r so far alternates between scal[8] and scal[9] (read one, write
// the other, `par` = iteration parity, so no workgroup sees this update's
// write); when r.r improves on it, the current v goes to vbest and the number
// of directions to flag[2]; once r.r exceeds DIVERGE2 times it, flag[0] = 4 and
// the host rolls the state back to that iterate.
constexpr double DIVERGE2 = 1e6;                 // a 1000-fold growth of the residual norm
// The two partial-sum arrays of the update (r.r of the previous iteration, d.w for eta),
// each summed in the fixed order of k_update2x's first version: thread t adds t, t + 256, ...
// then a tree over the 256 threads.  One workgroup per problem writes the totals to
// scal[12] and scal[13], which every workgroup of the update then reads.
constexpr int SCAL_RR = 12, SCAL_ETA = 13;
__global__ __launch_bounds__(256) void k_update_sums(const double* __restrict__ rr_in, int n_rr,
                                                     const double* __restrict__ eta_part, int n_eta,
                                                     double* __restrict__ scal, BatchStrides bs) {
  __shared__ double red[256], red2[256];
  {
    const i64 z = blockIdx.y;
    scal += z * bs.scal;
    if (eta_part) eta_part += z * bs.part;
    if (rr_in) rr_in += z * bs.part;
  }
  double pa = 0.0, pb = 0.0;
  if (rr_in)
    for (int i = threadIdx.x; i < n_rr; i += 256) pa += rr_in[i];
  if (eta_part)
    for (int i = threadIdx.x; i < n_eta; i += 256) pb += eta_part[i];
  red[threadIdx.x] = pa;
  red2[threadIdx.x] = pb;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) {
      red[threadIdx.x] += red[threadIdx.x + s2];
      red2[threadIdx.x] += red2[threadIdx.x + s2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[SCAL_RR] = red[0];
    scal[SCAL_ETA] = red2[0];
  }
}

// Small grids form the update's partial-sum totals inside every workgroup of k_update2x (one launch
// less per iteration: advection-diffusion 128^2 18.4 -> 18.0 ms per step); large ones once, in
// k_update_sums, where thousands of workgroups would each re-add them all (wave 64x128x128).
static bool update_inline(i64 N) { return (N + 255) / 256 <= 512; }

__global__ __launch_bounds__(256) void k_update2x(i64 N, const double* __restrict__ d, const double* __restrict__ w,
                                                  double* __restrict__ v, double* __restrict__ r,
                                                  double* __restrict__ X, double* __restrict__ Dcol,
                                                  double* __restrict__ Qcol, double* __restrict__ eta_slot,
                                                  double* __restrict__ scal, int* __restrict__ flag,
                                                  const double* __restrict__ eta_part, int n_eta,
                                                  const double* __restrict__ rr_in, int n_rr,
                                                  double* __restrict__ rr_out, BatchStrides bs,
                                                  double* __restrict__ vbest = nullptr, int par = 0,
                                                  int inl = 0) {
  __shared__ double red[256], red2[256];
  {                                              // problem blockIdx.y of a batch
    const i64 z = blockIdx.y;
    d += z * bs.v; w += z * bs.v; v += z * bs.v; r += z * bs.v; X += z * bs.v;
    Dcol += z * bs.M; Qcol += z * bs.M; eta_slot += z * bs.eta;
    scal += z * bs.scal; flag += z * bs.flag;
    if (rr_out) rr_out += z * bs.part;
    if (inl) {
      if (eta_part) eta_part += z * bs.part;
      if (rr_in) rr_in += z * bs.part;
    }
  }
  // every load of the update is issued up front: the flag, the totals and the vectors
  const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const int fl = flag[0];
  double dk = 0.0, wk = 0.0, vk = 0.0, rk0 = 0.0;
  if (k < N) {
    dk = d[k];
    wk = w[k];
    vk = v[k];
    rk0 = r[k];
  }
  // the totals of the partial sums: formed once by k_update_sums just before (inl = 0), or, for
  // small grids, by every workgroup itself in the same fixed order (the same bits, one launch less)
  double sr = rr_in ? scal[SCAL_RR] : scal[0];
  double et = eta_part ? scal[SCAL_ETA] : scal[1];
  const double stop2 = scal[4] * scal[3];
  if (inl && (rr_in || eta_part)) {
    double pa = 0.0, pb = 0.0;                 // thread t adds t, t + 256, ... in order
    if (rr_in)
      for (int i = threadIdx.x; i < n_rr; i += 256) pa += rr_in[i];
    if (eta_part)
      for (int i = threadIdx.x; i < n_eta; i += 256) pb += eta_part[i];
    red[threadIdx.x] = pa;
    red2[threadIdx.x] = pb;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if ((int)threadIdx.x < s2) {
        red[threadIdx.x] += red[threadIdx.x + s2];
        red2[threadIdx.x] += red2[threadIdx.x + s2];
      }
      __syncthreads();
    }
    if (rr_in) sr = red[0];
    if (eta_part) et = red2[0];
    __syncthreads();                           // red is reused for the r.r partials below
  }
  if (fl != 0) return;                         // uniform: every thread read the same flag
  if (rr_in && sr <= stop2) {
    if (k == 0) {
      scal[0] = sr;
      flag[0] = 1;
    }
    return;
  }
  if (vbest) {                                 // sr and the minimum are uniform over the grid
    const double rmin = scal[8 + par];
    if (sr > DIVERGE2 * rmin) {
      if (k == 0) {
        scal[0] = sr;
        flag[0] = 4;
      }
      return;
    }
    const bool better = sr < rmin;
    if (better && k < N) vbest[k] = vk;
    if (k == 0) {
      scal[9 - par] = better ? sr : rmin;
      if (better) flag[2] = flag[1];
    }
  }
  if (!(et > 0.0)) {
    if (k == 0) flag[0] = 2;
    return;
  }
  const double a = sr / et;
  double rr = 0.0;
  if (k < N) {
    v[k] = vk + a * dk;
    const double rk = rk0 - a * wk;
    r[k] = rk;
    X[k] = rk;
    Dcol[k] = dk;
    Qcol[k] = wk;
    rr = rk * rk;
  }
  if (k == 0) {
    *eta_slot = et;
    scal[0] = sr;
    scal[1] = et;
    flag[1] += 1;
  }
  if (rr_out) {
    rr = wave_sum(rr);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) rr_out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// r = b - y and X = r (guarded; problem blockIdx.y of a batch at offset blockIdx.y * vs, flags at * fs)
__global__ void k_resid2(i64 N, const double* __restrict__ b, const double* __restrict__ y, double* __restrict__ r,
                         double* __restrict__ X, const int* __restrict__ flag, i64 vs = 0, i64 fs = 0) {
  {
    const i64 z = blockIdx.y;
    b += z * vs; y += z * vs; r += z * vs; X += z * vs; flag += z * fs;
  }
  if (flag[0] != 0) return;
  const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) {
    const double v = b[k] - y[k];
    r[k] = v;
    X[k] = v;
  }
}

// guarded IterGP update of iteration slot `slot`
__global__ void k_update(i64 N, const double* __restrict__ d, double* __restrict__ v, double* __restrict__ Dcol,
                         double* __restrict__ eta_slot, const double* __restrict__ scal, int* __restrict__ flag) {
  const int state = flag[0];
  if (state != 0) return;
  const double et = scal[1], sr = scal[0];   // CG actions: s = r, so s.r = r.r
  if (!(et > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 2;   // breakdown: directions no longer S-definite
    return;
  }
  const double a = sr / et;
  const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) {
    const double dk = d[k];
    v[k] += a * dk;
    Dcol[k] = dk;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *eta_slot = et;
}

__global__ void k_count(int* flag, const double* scal) {
  if (flag[0] == 0 && scal[1] > 0.0) flag[1] += 1;
}

__global__ void k_sub_sq_acc(i64 M, int nr, const double* __restrict__ P, const double* __restrict__ Q,
                             const double* __restrict__ eta, double* __restrict__ acc) {
  const i64 x = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= M) return;
  double s = 0;
  for (int j = 0; j < nr; ++j) {
    const double w = P[(i64)j * M + x] - (Q ? Q[(i64)j * M + x] : 0.0);
    s += w * w / eta[j];
  }
  acc[x] += s;
}

// Column sums of squares of a rows x cols row-major block, added to acc.  The rows are split
// into gridDim.y chunks; a workgroup's four wavefronts take every fourth row of its chunk for
// 64 columns and meet in LDS (fixed order); k_colsq_finish adds the chunk partials in order.
__global__ __launch_bounds__(256) void k_colsq_part(i64 rows, i64 cols, const double* __restrict__ T,
                                                    double* __restrict__ part) {
  __shared__ double red[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const i64 c = (i64)blockIdx.x * 64 + lane;
  const i64 R = gridDim.y, ch = blockIdx.y;
  const i64 L = (rows + R - 1) / R, r0 = ch * L, r1 = min(rows, r0 + L);
  double s = 0.0;
  if (c < cols) {
#pragma unroll 8
    for (i64 r = r0 + wave; r < r1; r += 4) {
      const double t = T[r * cols + c];
      s = fma(t, t, s);
    }
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && c < cols) part[ch * cols + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ void k_colsq_finish(i64 cols, int R, const double* __restrict__ part, double* __restrict__ acc) {
  const i64 c = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int ch = 0; ch < R; ++ch) s += part[(i64)ch * cols + c];
  acc[c] += s;
}

constexpr int COLSQ_MAX_CHUNKS = 64;

// Row chunks for k_colsq_part: about 1024 workgroups in all
static int colsq_chunks(i64 rows, i64 cols) {
  const i64 colblocks = (cols + 63) / 64;
  const i64 want = (1024 + colblocks - 1) / colblocks;
  return (int)std::max<i64>(1, std::min<i64>({(i64)COLSQ_MAX_CHUNKS, want, rows}));
}

__global__ void k_var_final(i64 M, double sf2, const double* __restrict__ red, double* __restrict__ var) {
  const i64 x = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < M) var[x] = sf2 - red[x];
}

// dense point-grid cross-covariance block: out[b][x - x0] = sf2 prod_i P_i[b_i][x_i]
// Cross-covariances of the point observations with one output at the grid
// points: row b of group g is sum_c pc[g][c] prod_i P[g][c][i][b_i][x_i] over the
// group's components (pc = 0: a component on another output).
struct PGMeta {
  int d, ngroup;
  int gn[GPFVM_MAX_GROUPS][3];
  i64 goff[GPFVM_MAX_GROUPS + 1];
  int gdim[3];
  int gcomp[GPFVM_MAX_GROUPS];
  double pc[GPFVM_MAX_GROUPS][MAXC];               // outputscale x component coefficient
  const double* P[GPFVM_MAX_GROUPS][MAXC][3];      // n_{g,i} x G_i, component weights folded in
};

__global__ void k_point_grid(const PGMeta* __restrict__ meta, int nb, i64 x0, i64 nx,
                             double* __restrict__ out) {
  const PGMeta& G = *meta;
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (i64)nb * nx) return;
  const i64 b = idx / nx, xl = idx % nx, x = x0 + xl;
  int g = 0;
  while (g + 1 < G.ngroup && G.goff[g + 1] <= b) ++g;
  int ib[3] = {0, 0, 0}, ix[3] = {0, 0, 0};
  i64 r = b - G.goff[g];
  for (int i = G.d - 1; i >= 0; --i) { ib[i] = (int)(r % G.gn[g][i]); r /= G.gn[g][i]; }
  r = x;
  for (int i = G.d - 1; i >= 0; --i) { ix[i] = (int)(r % G.gdim[i]); r /= G.gdim[i]; }
  double v = 0.0;
  for (int c = 0; c < G.gcomp[g]; ++c) {
    if (G.pc[g][c] == 0.0) continue;
    double p = G.pc[g][c];
    for (int i = 0; i < G.d; ++i) p *= G.P[g][c][i][(i64)ib[i] * G.gdim[i] + ix[i]];
    v += p;
  }
  out[b * nx + xl] = v;
}


unsigned nblk(i64 n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// C[j][c] = (sum over the nch chunk partials in order) / eta[j] (eta null: no division)
__global__ void k_sum_rowscale(int nch, int rows, int cols, const double* __restrict__ part,
                               const double* __restrict__ eta, double* __restrict__ C) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  const i64 n = (i64)rows * cols;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[c * n + i];
  C[i] = eta ? s / eta[i / cols] : s;
}

// Plain CG (Sec. 4.1), device-side scalars: scal[CG_RR + (it & 1)] holds r.r of
// the current iteration, scal[CG_PAP] = p.S p, scal[3] = b.b, scal[4] = tol^2.
// flag[0]: 0 running, 1 converged, 2 breakdown (p.S p <= 0); flag[1]: updates made.
constexpr int CG_RR = 5, CG_PAP = 7;

// x += a p ; r -= a S p,  a = r.r / p.S p
__global__ void k_cg_step(i64 N, const double* __restrict__ p, const double* __restrict__ Sp, double* __restrict__ x,
                          double* __restrict__ r, const double* __restrict__ scal, int slot, int* __restrict__ flag) {
  if (flag[0] != 0) return;
  const double pap = scal[CG_PAP];
  if (!(pap > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 2;
    return;
  }
  const double a = scal[CG_RR + slot] / pap;
  const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) {
    x[k] += a * p[k];
    r[k] -= a * Sp[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) flag[1] += 1;
}

// stopping test on the new r.r, else p = r + (r.r_new / r.r) p
__global__ void k_cg_dir(i64 N, const double* __restrict__ r, double* __restrict__ p, const double* __restrict__ scal,
                         int slot, int* __restrict__ flag) {
  if (flag[0] != 0) return;
  const double rr = scal[CG_RR + slot], rn = scal[CG_RR + (slot ^ 1)];
  if (rn <= scal[4] * scal[3]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 1;
    return;
  }
  const double beta = rn / rr;
  const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) p[k] = r[k] + beta * p[k];
}

}  // namespace

GemmDesc gpfvm::desc1(void* C, i64 c_rs, const void* A, i64 a_rs, i64 a_cs, const void* B, i64 b_rs, i64 b_cs, int M,
               int N, int K, double alpha, double beta, int tri) {
  GemmDesc D;
  std::memset(&D, 0, sizeof(D));
  D.C = C; D.c_rs = c_rs; D.c_cs = 1; D.M = M; D.N = N; D.batch = 1; D.nseg = 1; D.beta = beta;
  Seg& S = D.seg[0];
  S.A = A; S.a_rs = a_rs; S.a_cs = a_cs; S.B = B; S.b_rs = b_rs; S.b_cs = b_cs; S.K = K; S.alpha = alpha;
  S.tri = tri;
  return D;
}


// ---------------------------------------------------------------------------
// G_bb^{-1} = L^{-T} L^{-1}, each triangular solve done as t = L^{-1} u
// followed by one correction t += L^{-1} (u - L t) (and likewise with L^T).
// Multiplying by an explicit inverse alone is not backward stable for this
// ill-conditioned block; the single residual correction restores it.
// Vectors are stored right-hand-side major (each a contiguous n_b vector).
// ---------------------------------------------------------------------------
std::vector<Stage> gpfvm::ginv_stages(const gpfvm_handle* h, int nrhs, const double* U, double* T, double* W,
                                      double* R) {
  const int nb = h->nb;
  std::vector<Stage> st(6);
  auto add = [&](int k, GemmDesc D) { st[k].descs.push_back(D); };
  // forward: T = Linv U ; R = U - L T ; T += Linv R     (B[j][i] = M[i][j], upper in (j, i))
  add(0, desc1(T, nb, U, nb, 1, h->Linv, 1, nb, nrhs, nb, nb, 1.0, 0.0, 3));
  {
    GemmDesc D = desc1(R, nb, T, nb, 1, h->L, 1, nb, nrhs, nb, nb, -1.0, 0.0, 3);
    D.X = U; D.x_rs = nb; D.x_cs = 1; D.gamma = 1.0;
    add(1, D);
  }
  add(2, desc1(T, nb, R, nb, 1, h->Linv, 1, nb, nrhs, nb, nb, 1.0, 1.0, 3));
  // backward: W = Linv^T T ; R = T - L^T W ; W += Linv^T R   (B[j][i] = M[j][i], lower)
  add(3, desc1(W, nb, T, nb, 1, h->Linv, nb, 1, nrhs, nb, nb, 1.0, 0.0, 4));
  {
    GemmDesc D = desc1(R, nb, W, nb, 1, h->L, nb, 1, nrhs, nb, nb, -1.0, 0.0, 4);
    D.X = T; D.x_rs = nb; D.x_cs = 1; D.gamma = 1.0;
    add(4, D);
  }
  add(5, desc1(W, nb, R, nb, 1, h->Linv, nb, 1, nrhs, nb, nb, 1.0, 1.0, 4));
  return st;
}

// y[i] = add[i] + alpha * sum_k M[i][k] x[k] over k <= i (upper = 0) or k >= i (upper = 1), for a
// row-major float64 or float32 matrix M, two adjacent rows per wavefront, so that each 16-byte load of x serves both
// rows (the loads of x come from L2 and had outnumbered the matrix's own: twice its bytes for a
// float32 matrix).  Matrix values in 16-byte loads (two float64 or four float32), UN of them per row
// in flight, products and sums in float64.  Needs n even (n % 4 == 0 for float32) and 16-byte
// aligned M and x.  The quads (pairs) inside both rows' ranges are shared; the up to 2V - 1 values
// of a row before them and after them are taken one by one by lanes 8 seg .. 8 seg + 7.
template <typename T, int UN>
__global__ __launch_bounds__(256) void k_trmv_2rows(int n, const T* __restrict__ M, const double* __restrict__ x,
                                                    double* __restrict__ y, double alpha,
                                                    const double* __restrict__ add, int upper) {
  constexpr int V = 16 / (int)sizeof(T);
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type VT;
  const int i0 = 2 * (blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (i0 >= n) return;                           // n is even: row i0 + 1 exists
  const int i1 = i0 + 1;
  const int lo0 = upper ? i0 : 0, hi0 = upper ? n : i0 + 1;
  const int lo1 = upper ? i1 : 0, hi1 = upper ? n : i1 + 1;
  const T* __restrict__ r0 = M + (i64)i0 * n;
  const T* __restrict__ r1 = r0 + n;
  const VT* __restrict__ v0 = reinterpret_cast<const VT*>(r0);
  const VT* __restrict__ v1 = reinterpret_cast<const VT*>(r1);
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);
  const int QA = max((lo0 + V - 1) / V, (lo1 + V - 1) / V), QB = min(hi0 / V, hi1 / V);
  auto dotv = [](const VT& m, const double2* xv) -> double {
    if constexpr (V == 2) return m.x * xv[0].x + m.y * xv[0].y;
    else return ((double)m.x * xv[0].x + (double)m.y * xv[0].y) + ((double)m.z * xv[1].x + (double)m.w * xv[1].y);
  };
  double a0 = 0.0, a1 = 0.0;
  if (QA < QB) {
    double c0[UN], c1[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) c0[u] = c1[u] = 0.0;
    int q = QA + lane;
    for (; q + 64 * (UN - 1) < QB; q += 64 * UN) {
      VT m0[UN], m1[UN];
      double2 xv[UN][V / 2];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        m0[u] = v0[q + 64 * u];
        m1[u] = v1[q + 64 * u];
#pragma unroll
        for (int hh = 0; hh < V / 2; ++hh) xv[u][hh] = x2[(q + 64 * u) * (V / 2) + hh];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        c0[u] += dotv(m0[u], xv[u]);
        c1[u] += dotv(m1[u], xv[u]);
      }
    }
    for (; q < QB; q += 64) {
      double2 xv[V / 2];
#pragma unroll
      for (int hh = 0; hh < V / 2; ++hh) xv[hh] = x2[q * (V / 2) + hh];
      c0[0] += dotv(v0[q], xv);
      c1[0] += dotv(v1[q], xv);
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      a0 += c0[u];
      a1 += c1[u];
    }
    // segments: 0 row i0 before the shared quads, 1 after them, 2 and 3 the same for row i1
    const int seg = lane >> 3, k = lane & 7;
    if (seg == 0 && lo0 + k < V * QA) a0 += (double)r0[lo0 + k] * x[lo0 + k];
    else if (seg == 1 && V * QB + k < hi0) a0 += (double)r0[V * QB + k] * x[V * QB + k];
    else if (seg == 2 && lo1 + k < V * QA) a1 += (double)r1[lo1 + k] * x[lo1 + k];
    else if (seg == 3 && V * QB + k < hi1) a1 += (double)r1[V * QB + k] * x[V * QB + k];
  } else {                                       // short rows (at most V values each)
    const int k = lane & 31;
    if (lane < 32) {
      if (lo0 + k < hi0) a0 = (double)r0[lo0 + k] * x[lo0 + k];
    } else if (lo1 + k < hi1) {
      a1 = (double)r1[lo1 + k] * x[lo1 + k];
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    y[i0] = (add ? add[i0] : 0.0) + alpha * a0;
    y[i1] = (add ? add[i1] : 0.0) + alpha * a1;
  }
}

template <typename T, int UN>
static hipError_t trmv_2rows(int n, const T* M, const double* x, double* y, double alpha, const double* add, int upper,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_trmv_2rows<T, UN>), dim3((unsigned)((n + 7) / 8)), dim3(256), 0, s, n, M, x, y, alpha, add,
                     upper);
  return hipGetLastError();
}

// Float32 copies of L^{-1} and L^{-T} for the correction products of the row-streaming solves
// (built once per handle; on allocation failure the corrections stay float64).
static void ensure_inv_f32(gpfvm_handle* h, hipStream_t s) {
  const i64 nn = (i64)h->nb * h->nb;
  if (!h->Linv_f) {
    float* p = (float*)h->arena.alloc((size_t)nn * sizeof(float));
    if (!p || launch_copy_f64_to_f32(h->Linv, p, nn, s) != hipSuccess) return;
    h->Linv_f = p;
  }
  if (!h->Linvt_f && h->Linvt) {
    float* p = (float*)h->arena.alloc((size_t)nn * sizeof(float));
    if (!p || launch_copy_f64_to_f32(h->Linvt, p, nn, s) != hipSuccess) return;
    h->Linvt_f = p;
  }
}

// float32 correction product (n % 4 == 0, M and x 16-byte aligned): two rows per wavefront, 100 us
// per pass over the 16384^2 float32 triangle against 114 us one row per wavefront
static hipError_t trmv_rows_f32(int n, const float* M, const double* x, double* y, double alpha, const double* add,
                                int upper, hipStream_t s) {
  return trmv_2rows<float, 2>(n, M, x, y, alpha, add, upper, s);
}

// float64 row-streaming product: two rows per wavefront where n is even and M and x are 16-byte
// aligned (188 us per pass over the 16384^2 float64 triangle, 5.7 TB/s, against 191 us one row per
// wavefront: this pass is bound by HBM, not by the loads of x), else one row per wavefront
static hipError_t trmv_rows_f64(int n, const double* M, const double* x, double* y, double alpha, const double* add,
                                int upper, hipStream_t s) {
  if (n % 2 == 0 && (uintptr_t)M % 16 == 0 && (uintptr_t)x % 16 == 0)
    return trmv_2rows<double, 4>(n, M, x, y, alpha, add, upper, s);
  return launch_trmv_rows(n, M, x, y, alpha, add, upper, s);
}

// Same six products for one right-hand side as row-streaming triangular
// matrix-vector products (large point blocks).  The two correction products
// L^{-1} r and L^{-T} r read float32 copies of the inverse when the handle has
// them: r is the residual of the first product, so the float32 rounding of
// the matrix (2^-24 relative) perturbs t and w by far less than float64
// rounding of the main products does, while the correction streams half the
// bytes.  The main products and the residuals stay float64.
hipError_t gpfvm::ginv_rows(const gpfvm_handle* h, const double* U, double* T, double* W, double* R, hipStream_t s) {
  const int nb = h->nb;
  const bool f32 = h->Linv_f && h->Linvt_f && nb % 4 == 0 && (uintptr_t)R % 16 == 0 && (uintptr_t)h->Linv_f % 16 == 0 &&
                   (uintptr_t)h->Linvt_f % 16 == 0;
  hipError_t e;
  if ((e = trmv_rows_f64(nb, h->Linv, U, T, 1.0, nullptr, 0, s)) != hipSuccess) return e;   // t = Li u
  if ((e = trmv_rows_f64(nb, h->L, T, R, -1.0, U, 0, s)) != hipSuccess) return e;           // r = u - L t
  e = f32 ? trmv_rows_f32(nb, h->Linv_f, R, T, 1.0, T, 0, s)                                // t += Li r
          : trmv_rows_f64(nb, h->Linv, R, T, 1.0, T, 0, s);
  if (e != hipSuccess) return e;
  if ((e = trmv_rows_f64(nb, h->Linvt, T, W, 1.0, nullptr, 1, s)) != hipSuccess) return e;  // w = Li^T t
  if ((e = trmv_rows_f64(nb, h->Lt, W, R, -1.0, T, 1, s)) != hipSuccess) return e;          // r = t - L^T w
  return f32 ? trmv_rows_f32(nb, h->Linvt_f, R, W, 1.0, W, 1, s)                            // w += Li^T r
             : trmv_rows_f64(nb, h->Linvt, R, W, 1.0, W, 1, s);
}

hipError_t gpfvm::run_stages(const std::vector<Stage>& st, hipStream_t s) {
  for (const Stage& x : st) {
    const hipError_t e = launch_gemm_stage(F64, x, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Q = L^{-1} G_bp (n_b x N, row-major), so that the point-block correction of
// the volume system is G_pb G_bb^{-1} G_bp = Q^T Q, symmetric by construction.
// G_bp comes from the closed-form Gram-entry kernel; the triangular solve is
// the explicit inverse with one residual correction, Q += L^{-1} (G_bp - L Q),
// which is backward stable where the inverse alone is not.
// ---------------------------------------------------------------------------
static int build_qc(gpfvm_handle* h, hipStream_t s) {
  if (h->Qc) return GPFVM_OK;
  const i64 N = h->N;
  const int nb = h->nb;
  const size_t bytes = (size_t)nb * N * sizeof(double);
  double* Q = (double*)h->arena.alloc(bytes);
  Arena tmp;
  tmp.cache = h->arena.cache;
  double* G = (double*)tmp.alloc(bytes);
  double* R = (double*)tmp.alloc(bytes);
  if (!Q || !G || !R) {
    tmp.release();
    h->err = "out of device memory (point correction Q)";
    return GPFVM_E_NOMEM;
  }
  hipError_t e = launch_gram_block(h->meta, 0, nb, nb, N, G, N, s);
  std::vector<Stage> st(3);
  st[0].descs.push_back(desc1(Q, N, h->Linv, nb, 1, G, N, 1, nb, (int)N, nb, 1.0, 0.0, 1));
  {
    GemmDesc D = desc1(R, N, h->L, nb, 1, Q, N, 1, nb, (int)N, nb, -1.0, 0.0, 1);
    D.X = G; D.x_rs = N; D.x_cs = 1; D.gamma = 1.0;
    st[1].descs.push_back(D);
  }
  st[2].descs.push_back(desc1(Q, N, h->Linv, nb, 1, R, N, 1, nb, (int)N, nb, 1.0, 1.0, 1));
  if (e == hipSuccess) e = upload_stages(st, tmp, s);
  if (e == hipSuccess) e = run_stages(st, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  tmp.release();
  if (e != hipSuccess || e2 != hipSuccess) {
    h->err = std::string("building the point correction Q failed: ") + hipGetErrorString(e != hipSuccess ? e : e2);
    return GPFVM_E_HIP;
  }
  h->Qc = Q;
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// Factored point correction (2-D, every point group pinned in one dimension,
// no per-cell coefficients).  Piece r = (group g, PDE term t): the group's
// cross-covariance with the volumes is sf2 coef_t Gf (x) q over its free and
// pinned dimensions (the point-cell factors of Sec. 3.2), so G_bp =
// sum_r Gf_r (x)_{p_r} q_r.  Then M_cat = L^{-1} [Gf_0 | Gf_1 | ...] (the
// explicit inverse with one residual correction, as for Q) and P = M_cat^T
// M_cat give Q^T Q x = sum_r q_r (x) (P w)_r with n_b W + W^2 work in place
// of the n_b N of a resident Q.
// ---------------------------------------------------------------------------
static bool qfact_ok(const gpfvm_handle* h, int* W_out, int* R_out) {
  if (h->d != 2 || h->nb <= 0 || h->multi) return false;
  for (const auto& t : h->pterms)
    if (t.cellwise) return false;
  int W = 0, R = 0;
  for (const auto& G : h->groups) {
    if (G.n[0] != 1 && G.n[1] != 1) return false;
    const int f = G.n[0] == 1 ? 1 : 0;
    for (size_t t = 0; t < h->pterms.size(); ++t) {
      W += h->nc[f];
      ++R;
    }
  }
  if (R < 1 || R > QF_MAXR || W > QF_MAXW) return false;
  *W_out = W;
  *R_out = R;
  return true;
}

static int build_qf(gpfvm_handle* h, hipStream_t s) {
  if (h->qf) return GPFVM_OK;
  int W = 0, R = 0;
  if (!qfact_ok(h, &W, &R)) { h->err = "factored point correction: not applicable"; return GPFVM_E_INVALID; }
  const int nb = h->nb, n0 = h->nc[0], n1 = h->nc[1];
  QFactor F;
  F.R = R; F.W = W; F.n0 = n0; F.n1 = n1;
  F.nunit = 0;
  std::vector<double> gf((size_t)nb * W, 0.0), fac;
  std::vector<std::vector<double>> qh;                  // host copies of the q_r
  HIPCHK(h, hipStreamSynchronize(s));                    // the point-cell factors are complete
  int r = 0, off = 0;
  for (int pass = 0; pass < 2; ++pass)                   // pieces pinned in dimension 0 first
    for (size_t gi = 0; gi < h->groups.size(); ++gi) {
      const Group& G = h->groups[gi];
      const int p = G.n[0] == 1 ? 0 : 1, f = 1 - p;
      if (p != pass) continue;
      const int nf = G.n[f], cf = h->nc[f];
      for (size_t ti = 0; ti < h->pterms.size(); ++ti, ++r) {
        F.p[r] = p;
        F.off[r] = off;
        F.q[r] = h->Qfac[gi][ti][p].d;                   // 1 x nc[p]
        F.nunit += (cf + QF_UW - 1) / QF_UW;
        qh.emplace_back((size_t)h->nc[p]);
        HIPCHK(h, hipMemcpy(qh.back().data(), F.q[r], qh.back().size() * sizeof(double), hipMemcpyDeviceToHost));
        fac.resize((size_t)nf * cf);
        HIPCHK(h, hipMemcpy(fac.data(), h->Qfac[gi][ti][f].d, fac.size() * sizeof(double), hipMemcpyDeviceToHost));
        const double a = h->sf2 * h->pterms[ti].coef;
        for (int k = 0; k < nf; ++k)
          for (int c = 0; c < cf; ++c) gf[(size_t)(G.offset + k) * W + off + c] = a * fac[(size_t)k * cf + c];
        off += cf;
      }
    }
  // the constant operands of the last-stage segments
  const int nu = F.nunit;
  int R0 = 0;
  while (R0 < R && F.p[R0] == 0) ++R0;
  const int K0 = R0 * nu, K1 = (R - R0) * nu;
  F.w0 = R0 * n1;
  std::vector<double> aq((size_t)n0 * std::max(K0, 1), 0.0), bq((size_t)std::max(K1, 1) * n1, 0.0);
  for (int rr = 0; rr < R0; ++rr)
    for (int u = 0; u < nu; ++u)
      for (int i = 0; i < n0; ++i) aq[(size_t)i * K0 + rr * nu + u] = qh[rr][i];
  for (int rr = R0; rr < R; ++rr)
    for (int u = 0; u < nu; ++u)
      for (int c = 0; c < n1; ++c) bq[(size_t)((rr - R0) * nu + u) * n1 + c] = qh[rr][c];
  double* P = (double*)h->arena.alloc((size_t)W * W * sizeof(double));
  QFactor* Fd = (QFactor*)h->arena.alloc(sizeof(QFactor));
  double* Aq = (double*)h->arena.alloc(aq.size() * sizeof(double));
  double* Bq = (double*)h->arena.alloc(bq.size() * sizeof(double));
  Arena tmp;
  tmp.cache = h->arena.cache;
  const size_t bytes = (size_t)nb * W * sizeof(double);
  double* Gd = (double*)tmp.alloc(bytes);
  double* M = (double*)tmp.alloc(bytes);
  double* Rr = (double*)tmp.alloc(bytes);
  if (!P || !Fd || !Aq || !Bq || !Gd || !M || !Rr) {
    tmp.release();
    h->err = "out of device memory (factored point correction)";
    return GPFVM_E_NOMEM;
  }
  F.P = P;
  hipError_t e = hipMemcpyAsync(Gd, gf.data(), bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(Fd, &F, sizeof(QFactor), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(Aq, aq.data(), aq.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(Bq, bq.data(), bq.size() * sizeof(double), hipMemcpyHostToDevice, s);
  std::vector<Stage> st(4);
  st[0].descs.push_back(desc1(M, W, h->Linv, nb, 1, Gd, W, 1, nb, W, nb, 1.0, 0.0, 1));
  {
    GemmDesc D = desc1(Rr, W, h->L, nb, 1, M, W, 1, nb, W, nb, -1.0, 0.0, 1);
    D.X = Gd; D.x_rs = W; D.x_cs = 1; D.gamma = 1.0;
    st[1].descs.push_back(D);
  }
  st[2].descs.push_back(desc1(M, W, h->Linv, nb, 1, Rr, W, 1, nb, W, nb, 1.0, 1.0, 1));
  st[3].descs.push_back(desc1(P, W, M, 1, W, M, W, 1, W, W, nb, 1.0, 0.0, 0));   // P = M^T M
  if (e == hipSuccess) e = upload_stages(st, tmp, s);
  if (e == hipSuccess) e = run_stages(st, s);
  const hipError_t e2 = hipStreamSynchronize(s);          // gf, F, aq and bq are host buffers
  tmp.release();
  if (e != hipSuccess || e2 != hipSuccess) {
    h->err = std::string("building the factored point correction failed: ") +
             hipGetErrorString(e != hipSuccess ? e : e2);
    return GPFVM_E_HIP;
  }
  h->qf = Fd;
  h->qf_nunit = nu;
  h->qf_w0 = R0 * n1;
  h->qf_k0 = K0;
  h->qf_k1 = K1;
  h->qf_aq = Aq;
  h->qf_bq = Bq;
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// volume-system operator S for nrhs right-hand sides.  elt = F32 gives the
// mixed operator: the volume Kronecker block in float32 (float32 factors,
// float32 accumulation), the point-block correction in float64.
// ---------------------------------------------------------------------------
int gpfvm::get_sop(gpfvm_handle* h, int nrhs, Elt elt, gpfvm_sop** out) {
  auto& tab = (elt == F64) ? h->sops : h->sops32;
  auto it = tab.find(nrhs);
  if (it != tab.end()) { *out = it->second.get(); return GPFVM_OK; }
  if (elt != F64 && h->multi) { h->err = "the mixed path takes single-output problems"; return GPFVM_E_INVALID; }
  if (elt != F64 && h->op_pp32.empty()) {
    int rc = build_ops32(h);
    if (rc) return rc;
  }
  // the low-precision volume plan: float32 MFMA, or split-bfloat16 MFMA (float32 storage)
  const Elt lowp = h->tile == GPFVM_TILE_BF16X3 ? F32B : F32;
  auto so = std::make_unique<gpfvm_sop>();
  so->nrhs = nrhs;
  so->elt = elt;
  const i64 N = h->N, nb = std::max(h->nb, 1);
  so->X = h->arena.alloc((size_t)N * nrhs * 8);
  so->Y = h->arena.alloc((size_t)N * nrhs * 8);
  so->U = h->arena.alloc((size_t)nb * nrhs * 8);
  so->T = h->arena.alloc((size_t)nb * nrhs * 8);
  so->W = h->arena.alloc((size_t)nb * nrhs * 8);
  so->R = h->arena.alloc((size_t)nb * nrhs * 8);
  if (!so->X || !so->Y || !so->U || !so->T || !so->W || !so->R) {
    h->err = "out of device memory (S operator)";
    return GPFVM_E_NOMEM;
  }
  int rc;
  if (elt == F64) {
    rc = compile_kron_list(h->op_pp, F64, nrhs, so->X, N, so->Y, N, h->cellc, h->cellc, 0.0, so->X, h->sig_pde,
                           pp_accumulate(h), h->arena, h->stream, so->pp, h->err);
  } else {
    so->X32 = h->arena.alloc((size_t)N * nrhs * 4);
    so->Y32 = h->arena.alloc((size_t)N * nrhs * 4);
    if (!so->X32 || !so->Y32) { h->err = "out of device memory (S operator)"; return GPFVM_E_NOMEM; }
    rc = compile_kron_list(h->op_pp32, lowp, nrhs, so->X32, N, so->Y32, N, h->cellc_f, h->cellc, 0.0, so->X32, h->sig_pde,
                           1, h->arena, h->stream, so->pp, h->err);
  }
  if (rc) return rc;
  so->flops_pp = so->pp.flops;
  if (h->nb > 0) {
    rc = compile_kron_list(h->op_bp, F64, nrhs, so->X, N, so->U, h->nb, h->cellc, h->cellc, 0.0, nullptr, 0, 0,
                           h->arena, h->stream, so->bp, h->err);
    if (rc) return rc;
    std::vector<KronOp> pb = h->op_pb;
    for (auto& o : pb)
      for (auto& t : o.terms) t.alpha = -t.alpha;
    rc = compile_kron_list(pb, F64, nrhs, so->W, h->nb, so->Y, N, h->cellc, h->cellc, 1.0, nullptr, 0, 1, h->arena,
                           h->stream, so->pb, h->err);
    if (rc) return rc;
    so->ginv = ginv_stages(h, nrhs, (const double*)so->U, (double*)so->T, (double*)so->W, (double*)so->R);
    if (upload_stages(so->ginv, h->arena, h->stream, F64) != hipSuccess) {
      h->err = "descriptor check/upload failed";
      return GPFVM_E_HIP;
    }
    so->ginv_small = (nrhs == 1 && h->nb <= SMALL_GINV_MAX && h->Lt && h->Linvt);
    // the factored form needs the 2-D volume operator's last stage as one descriptor over the
    // row-major n0 x n1 output, with room for two more segments
    int qW = 0, qR = 0;
    bool qf_fit = elt == F64 && nrhs == 1 && qform_ok(N, h->nb) && so->pp.stages.size() >= 2 &&
                  qfact_ok(h, &qW, &qR);
    if (qf_fit) {
      const Stage& L = so->pp.stages.back();
      const GemmDesc& D = L.descs.empty() ? GemmDesc() : L.descs[0];
      qf_fit = L.descs.size() == 1 && D.M == h->nc[0] && D.N == h->nc[1] && D.batch == 1 &&
               D.c_rs == h->nc[1] && D.c_cs == 1 && D.nseg + 2 <= MAXSEG && L.rider.kind == RIDE_NONE &&
               so->pp.stages.front().rider.kind == RIDE_NONE;
    }
    if (qf_fit) {
      rc = build_qf(h, h->stream);
      if (rc) return rc;
      so->qform = so->qf = true;
      const int nu = h->qf_nunit, n0 = h->nc[0], n1 = h->nc[1];
      so->qf_v = (double*)h->arena.alloc((size_t)nu * qW * sizeof(double));
      if (!so->qf_v) { h->err = "out of device memory (S operator)"; return GPFVM_E_NOMEM; }
      so->pp_split = so->pp;
      // the partial sums of v = P w(X) ride on the first stage (it reads X only)
      Rider& r1 = so->pp_split.stages.front().rider;
      r1.kind = RIDE_QFV;
      r1.nr = nu;
      r1.N = N;
      r1.v = (const double*)so->X;
      r1.out = so->qf_v;
      r1.qf = h->qf;
      // Y -= sum_r q_r (x) v_r as two more segments of the last stage
      std::vector<Stage> last{so->pp_split.stages.back()};
      GemmDesc& D = last[0].descs[0];
      if (h->qf_k0 > 0) {
        Seg& S = D.seg[D.nseg++];
        std::memset(&S, 0, sizeof(S));
        S.A = h->qf_aq; S.a_rs = h->qf_k0; S.a_cs = 1;
        S.B = so->qf_v; S.b_rs = n1; S.b_cs = 1;
        S.K = h->qf_k0; S.alpha = -1.0;
      }
      if (h->qf_k1 > 0) {
        Seg& S = D.seg[D.nseg++];
        std::memset(&S, 0, sizeof(S));
        S.A = so->qf_v + (size_t)nu * h->qf_w0; S.a_rs = 1; S.a_cs = n0;
        S.B = h->qf_bq; S.b_rs = n1; S.b_cs = 1;
        S.K = h->qf_k1; S.alpha = -1.0;
      }
      if (upload_stages(last, h->arena, h->stream, F64) != hipSuccess) {
        h->err = "descriptor check/upload failed";
        return GPFVM_E_HIP;
      }
      so->pp_split.stages.back() = last[0];
    } else if (elt != F64 && nrhs == 1 && qform_ok(N, h->nb)) {
      // low-precision operator: the resident Q applied on its own around the volume plan
      rc = build_qc(h, h->stream);
      if (rc) return rc;
      so->qform = true;
    } else if (elt == F64 && nrhs == 1 && qform_ok(N, h->nb)) {
      rc = build_qc(h, h->stream);
      if (rc) return rc;
      so->qform = true;
      // U = Q X rides in the launch of the volume operator's first stage (both read X only)
      if (!so->pp.stages.empty()) {
        Rider& rd = so->pp.stages[0].rider;
        rd.kind = RIDE_ROWS;
        rd.nr = (int)h->nb;
        rd.N = N;
        rd.M = h->Qc;
        rd.v = (const double*)so->X;
        rd.eta = nullptr;
        rd.out = (double*)so->U;
      }
      // split form for the two-pass loop: Q^T U also rides, on the last stage (U is complete by then)
      if (so->pp.stages.size() >= 2) {
        so->csub = (double*)h->arena.alloc((size_t)N * sizeof(double));
        if (!so->csub) { h->err = "out of device memory (S operator)"; return GPFVM_E_NOMEM; }
        so->pp_split = so->pp;
        Rider& rc2 = so->pp_split.stages.back().rider;
        rc2.kind = RIDE_COLS;
        rc2.nr = (int)h->nb;
        rc2.N = N;
        rc2.M = h->Qc;
        rc2.v = (const double*)so->U;
        rc2.eta = nullptr;
        rc2.out = so->csub;
        so->split = true;
      }
    }
  }
  // the one-rhs row-streaming point solve reads float32 copies of the inverse for its corrections
  if (elt == F64 && nrhs == 1 && h->nb > 0 && !so->ginv_small && !so->qform && !so->qf) ensure_inv_f32(h, h->stream);
  if (elt == F64) {
    std::vector<const Plan*> parts{&so->pp};
    if (h->nb > 0) parts.push_back(&so->bp);
    rc = merge_plans(parts, h->arena, h->stream, so->front, h->err);
    if (rc) return rc;
  }
  *out = so.get();
  tab[nrhs] = std::move(so);
  return GPFVM_OK;
}

// W = G_bb^{-1} U on the operator's bound buffers
static hipError_t apply_ginv(gpfvm_handle* h, gpfvm_sop* so, hipStream_t s) {
  if (so->ginv_small)
    return launch_ginv_small(h->nb, h->L, h->Linv, h->Lt, h->Linvt, (const double*)so->U, (double*)so->W, s);
  if (so->nrhs == 1) return ginv_rows(h, (const double*)so->U, (double*)so->T, (double*)so->W, (double*)so->R, s);
  return run_stages(so->ginv, s);
}

// Y = S X on the operator's bound buffers (X, Y float64; X32 filled by the caller for F32)
static hipError_t apply_sop(gpfvm_handle* h, gpfvm_sop* so, hipStream_t s) {
  hipError_t e;
  const i64 NN = h->N * so->nrhs;
  if (so->qf) return run_plan(so->pp_split, s);             // G_pp X + s2 X - sum_r q_r (x) (P w)_r
  if (so->qform && so->elt != F64) {                                // low-precision G_pp, float64 Q^T Q X
    if ((e = launch_rows_dot_full(h->nb, h->N, h->Qc, (const double*)so->X, (double*)so->U, s)) != hipSuccess) return e;
    if ((e = launch_copy_f64_to_f32((const double*)so->X, (float*)so->X32, NN, s)) != hipSuccess) return e;
    if ((e = run_plan(so->pp, s)) != hipSuccess) return e;
    if ((e = launch_copy_f32_to_f64((const float*)so->Y32, (double*)so->Y, NN, s)) != hipSuccess) return e;
    return launch_cols_update(h->nb, h->N, h->Qc, (double*)so->U, 1, nullptr, (const double*)so->Y,
                              (double*)so->Y, nullptr, nullptr, nullptr, nullptr, s);
  }
  if (so->qform) {                                                  // G_pp X + s2 X - Q^T Q X
    if (so->pp.stages.empty() &&
        (e = launch_rows_dot_full(h->nb, h->N, h->Qc, (const double*)so->X, (double*)so->U, s)) != hipSuccess)
      return e;
    if ((e = run_plan(so->pp, s)) != hipSuccess) return e;               // (with U = Q X riding along)
    return launch_cols_update(h->nb, h->N, h->Qc, (double*)so->U, 1, nullptr, (const double*)so->Y,
                              (double*)so->Y, nullptr,
                              nullptr, nullptr, nullptr, s);
  }
  if (so->elt == F64) {
    if ((e = run_plan(so->front, s)) != hipSuccess) return e;      // G_pp X + s2 X  and  G_bp X
  } else {
    if ((e = launch_copy_f64_to_f32((const double*)so->X, (float*)so->X32, NN, s)) != hipSuccess) return e;
    if ((e = run_plan(so->pp, s)) != hipSuccess) return e;
    if ((e = launch_copy_f32_to_f64((const float*)so->Y32, (double*)so->Y, NN, s)) != hipSuccess) return e;
    if (h->nb > 0 && (e = run_plan(so->bp, s)) != hipSuccess) return e;
  }
  if (h->nb > 0) {
    if ((e = apply_ginv(h, so, s)) != hipSuccess) return e;
    if ((e = run_plan(so->pb, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// y = S x for one float64 vector (through the float64 or the mixed operator)
static int apply_S(gpfvm_handle* h, Elt elt, const double* x, double* y, hipStream_t s) {
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, 1, elt, &so);
  if (rc) return rc;
  const i64 N = h->N;
  HIPCHK(h, hipMemcpyAsync(so->X, x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, apply_sop(h, so, s));
  HIPCHK(h, hipMemcpyAsync(y, so->Y, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  return GPFVM_OK;
}

extern "C" int gpfvm_schur_matvec(gpfvm_handle* h, int nrhs, const double* x, double* y, int prec, void* stream) {
  if (!h) return GPFVM_E_INVALID;
  if (nrhs < 1 || nrhs > 4096 || !x || !y) { h->err = "schur_matvec: bad nrhs or NULL buffer"; return GPFVM_E_INVALID; }
  if (prec != GPFVM_PREC_FP64 && prec != GPFVM_PREC_MIXED) { h->err = "schur_matvec: bad prec"; return GPFVM_E_INVALID; }
  const size_t bytes = (size_t)h->N * nrhs * sizeof(double);
  if ((const char*)x < (const char*)y + bytes && (const char*)y < (const char*)x + bytes) {
    h->err = "schur_matvec: x and y overlap";
    return GPFVM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, nrhs, prec == GPFVM_PREC_FP64 ? F64 : F32, &so);
  if (rc) return rc;
  HIPCHK(h, hipMemcpyAsync(so->X, x, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, apply_sop(h, so, s));
  HIPCHK(h, hipMemcpyAsync(y, so->Y, bytes, hipMemcpyDeviceToDevice, s));
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// solver state
// ---------------------------------------------------------------------------
static int ensure_state(gpfvm_handle* h, hipStream_t s) {
  if (h->v) return GPFVM_OK;
  const i64 N = h->N;
  h->bS = (double*)h->arena.alloc(N * sizeof(double));
  h->ab0 = (double*)h->arena.alloc(std::max(h->nb, 1) * sizeof(double));
  h->v = (double*)h->arena.alloc(N * sizeof(double));
  h->Dd = (double*)h->arena.alloc((size_t)N * h->max_iter * sizeof(double));
  h->eta = (double*)h->arena.alloc(h->max_iter * sizeof(double));
  h->vec = (double*)h->arena.alloc((size_t)8 * N * sizeof(double));
  // 1024 dot partials, then the row-dot partials of the projections and the column update's
  // finished coefficients after them (<= 2 max_iter + ROWS_DOT_TARGET - 1)
  h->aux = (double*)h->arena.alloc((size_t)(1024 + ROWS_DOT_TARGET + 2 * h->max_iter) * sizeof(double));
  h->scal = (double*)h->arena.alloc(64 * sizeof(double));
  h->flag = (int*)h->arena.alloc(16 * sizeof(int));
  h->part = (double*)h->arena.alloc((size_t)((N + 63) / 64 + 2 * nblk(N) + 1) * sizeof(double));
  if (!h->bS || !h->ab0 || !h->v || !h->Dd || !h->eta || !h->vec || !h->aux || !h->scal || !h->flag || !h->part) {
    h->err = "out of device memory (solver state; lower max_iter)";
    return GPFVM_E_NOMEM;
  }
  // b = y_p - G_pb G_bb^{-1} y_b ; ab0 = G_bb^{-1} y_b
  HIPCHK(h, hipMemcpyAsync(h->bS, h->yobs + h->nb, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h->nb > 0) {
    gpfvm_sop* so = nullptr;
    int rc = get_sop(h, 1, F64, &so);
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(so->U, h->yobs, h->nb * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, run_stages(so->ginv, s));
    HIPCHK(h, hipMemcpyAsync(h->ab0, so->W, h->nb * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the volume plan of S accumulates -G_pb W into Y (beta = 1): start from zero
    HIPCHK(h, launch_fill((double*)so->Y, 0.0, N, s));
    HIPCHK(h, run_plan(so->pb, s));
    HIPCHK(h, launch_axpby(N, 1.0, (const double*)so->Y, 1.0, h->bS, s));
  }
  return GPFVM_OK;
}

// One IterGP run on the volume system with right-hand side `b`, float64
// recurrences, operator precision `elt`.  Directions are appended from slot
// `start`; v accumulates.  passes = 1 is the published recurrence
// d = s - C z with eta = z^T d and an explicit residual every iteration.
// passes = 2 projects twice (classical Gram-Schmidt twice in the S inner
// product) with one operator application per iteration: z = S s; first pass
// c = eta^-1 o D^T z, d = s - D c, w = z - (S D) c (= S d); second pass
// c = eta^-1 o D^T w, d -= D c, w -= (S D) c; then eta = d^T w, S D gains w,
// and the residual is updated recursively with w and replaced by b - S v
// every `replace_every` iterations.  The operator's input buffer X doubles as
// the action vector, so no vector is copied inside the loop.
static int itergp_run(gpfvm_handle* h, Elt elt, const double* b, double* v, int start, int max_new, double tol,
                      int check_every, int passes, int replace_every, hipStream_t s, int* n_out, int* state_out,
                      const std::function<int(int)>* action = nullptr, bool res64 = false) {
  const i64 N = h->N;
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, 1, elt, &so);
  if (rc) return rc;
  double* X = (double*)so->X;
  const double* Y = (const double*)so->Y;
  double* r = h->vec;
  double* d = h->vec + 2 * N;
  double* w = h->vec + 5 * N;
  double* dotp = h->aux;              // 512 dot partials
  double* coef = h->aux + 1024;       // row-dot partials of D^T (.) for the projections
  if (passes == 2 && !h->Qd) {
    h->Qd = (double*)h->arena.alloc((size_t)N * h->max_iter * sizeof(double));
    if (!h->Qd) { h->err = "out of device memory (S D store; lower max_iter)"; return GPFVM_E_NOMEM; }
  }
  const int end = std::min(h->max_iter, start + max_new);
  // r = b - S v ; X = r   (res64: S in float64 whatever the loop's operator, the
  // refinement residual of the mixed-precision blocks)
  HIPCHK(h, hipMemsetAsync(h->flag, 0, 16 * sizeof(int), s));
  const double* Y0 = Y;
  if (res64 && elt != F64) {
    double* y64 = h->vec + 6 * N;
    rc = apply_S(h, F64, v, y64, s);
    if (rc) return rc;
    Y0 = y64;
  } else {
    HIPCHK(h, hipMemcpyAsync(X, v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, apply_sop(h, so, s));
  }
  HIPCHK(h, launch_dot(N, b, b, dotp, h->scal + 3, s));
  {
    const double t2 = action ? -1.0 : tol * tol;     // caller's actions: no stopping test
    HIPCHK(h, hipMemcpyAsync(h->scal + 4, &t2, sizeof(double), hipMemcpyHostToDevice, s));
    static const double inf2[2] = {HUGE_VAL, HUGE_VAL};   // the divergence guard's smallest r.r
    HIPCHK(h, hipMemcpyAsync(h->scal + 8, inf2, sizeof(inf2), hipMemcpyHostToDevice, s));
  }
  // the divergence guard (two-pass loop with CG actions): v at the smallest residual
  double* vbest = (passes == 2 && !action) ? h->vec + 7 * N : nullptr;
  hipLaunchKernelGGL(k_resid2, dim3(nblk(N)), dim3(256), 0, s, N, b, Y0, r, X, (const int*)h->flag);
  int i = start;
  int hflag[3] = {0, 0, 0};
  // coef = partial sums of D^T rhs over the first nd stored directions; the column update adds
  // them up and divides by eta, so it applies eta^-1 o (D^T rhs)
  auto project = [&](const double* rhs_vec, int nd) {
    return launch_rows_dot(nd, N, h->Dd, rhs_vec, coef, s);
  };
  // two-pass form: r.r and the stopping test of an iteration come from the
  // previous update's partial sums (tested inside the update kernel), or from
  // the dot kernel at the start and after an explicit residual replacement
  const int n_eta = (int)((N + 63) / 64), n_rr = (int)nblk(N);
  const bool upd_inl = update_inline(N);
  double* eta_p = h->part;
  double* rr_a = h->part + n_eta;
  double* rr_b = rr_a + n_rr;
  double* rr_prev = nullptr;
  if (passes == 2) HIPCHK(h, launch_dot_check(N, r, dotp, h->scal, h->flag, end - start, s));
  // Iterations run in batches between host checks of the flags.  The batch
  // length is check_every, shortened near convergence to the number of
  // iterations the residual's geometric rate over the last batch predicts
  // (plus one), so few iterations run after the stopping test has fired.
  int batch = std::max(1, check_every);
  double rr_last = -1.0;
  int i_last = i;
  while (i < end) {
    const int batch_end = std::min(end, i + batch);
    for (; i < batch_end; ++i) {
      // scal[0] = r.r and the stopping test; s = r is already in X
      if (passes == 1) HIPCHK(h, launch_dot_check(N, r, dotp, h->scal, h->flag, end - start, s));
      if (action) {                                           // s = the caller's action (in X)
        const int rc = (*action)(i);
        if (rc) return rc;
      }
      // z = S s: in Y, or as Y - csub with the split Q-form (two-pass loop)
      const bool split = (passes == 2 && so->split);
      if (split) HIPCHK(h, run_plan(so->pp_split, s));
      else HIPCHK(h, apply_sop(h, so, s));
      const double* zm = split ? so->csub : nullptr;
      if (passes == 1) {
        HIPCHK(h, hipMemcpyAsync(h->vec + N, Y, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (i > 0) {                                          // d = s - D (eta^-1 o D^T z)
          HIPCHK(h, project(Y, i));
          HIPCHK(h, launch_cols_update(i, N, h->Dd, coef, rows_dot_chunks(i, N), h->eta, X, d, X, nullptr, nullptr,
                                       nullptr, s));
        } else {
          HIPCHK(h, hipMemcpyAsync(d, X, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
      } else {
        if (i > 0) {
          // first pass: c = eta^-1 o D^T z ; d = s - D c ; w = S d = z - (S D) c
          HIPCHK(h, launch_rows_dot(i, N, h->Dd, Y, coef, s, zm));
          HIPCHK(h, launch_cols_update(i, N, h->Dd, coef, rows_dot_chunks(i, N), h->eta, X, d, nullptr, h->Qd, Y, w,
                                       s, nullptr, zm));
          // second pass on (d, w): c = eta^-1 o D^T w ; d -= D c ; w -= (S D) c ; eta = d^T w
          HIPCHK(h, project(w, i));
          HIPCHK(h, launch_cols_update(i, N, h->Dd, coef, rows_dot_chunks(i, N), h->eta, d, d, nullptr, h->Qd, w, w,
                                       s, eta_p));
        } else {
          HIPCHK(h, hipMemcpyAsync(d, X, N * sizeof(double), hipMemcpyDeviceToDevice, s));
          HIPCHK(h, hipMemcpyAsync(w, Y, N * sizeof(double), hipMemcpyDeviceToDevice, s));
          if (zm) HIPCHK(h, launch_axpby(N, -1.0, zm, 1.0, w, s));   // w = z = Y - csub
          HIPCHK(h, launch_dot(N, w, d, dotp, h->scal + 1, s));   // eta = d^T S d
        }
      }
      if (passes == 2) {
        const bool replace = (i + 1 - start) % std::max(1, replace_every) == 0;
        double* rr_next = (replace || action) ? nullptr : (rr_prev == rr_a ? rr_b : rr_a);
        // with CG actions s = r, so the step numerator s^T r is r^T r; otherwise d^T r
        if (action) HIPCHK(h, launch_dot(N, d, r, dotp, h->scal, s));
        if (!upd_inl && (i > 0 || rr_prev))
          hipLaunchKernelGGL(k_update_sums, dim3(1), dim3(256), 0, s, (const double*)rr_prev, n_rr,
                             (const double*)(i > 0 ? eta_p : nullptr), n_eta, h->scal, BatchStrides());
        hipLaunchKernelGGL(k_update2x, dim3(nblk(N)), dim3(256), 0, s, N, (const double*)d, (const double*)w, v, r,
                           X, h->Dd + (i64)i * N, h->Qd + (i64)i * N, h->eta + i, h->scal, h->flag,
                           (const double*)(i > 0 ? eta_p : nullptr), n_eta, (const double*)rr_prev, n_rr, rr_next,
                           BatchStrides(), vbest, (i - start) & 1, upd_inl ? 1 : 0);
        rr_prev = rr_next;
        if (replace) {
          HIPCHK(h, hipMemcpyAsync(X, v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
          HIPCHK(h, apply_sop(h, so, s));
          hipLaunchKernelGGL(k_resid2, dim3(nblk(N)), dim3(256), 0, s, N, b, Y, r, X, (const int*)h->flag);
          // X must hold r again even when the run has already stopped
          HIPCHK(h, hipMemcpyAsync(X, r, N * sizeof(double), hipMemcpyDeviceToDevice, s));
          HIPCHK(h, launch_dot_check(N, r, dotp, h->scal, h->flag, end - start, s));
        }
      } else {
        // eta = z^T d with z = S s: recompute z is not needed -- z was in Y before the
        // projection; the one-pass recurrence keeps a copy of it
        HIPCHK(h, launch_dot(N, h->vec + N, d, dotp, h->scal + 1, s));
        hipLaunchKernelGGL(k_update, dim3(nblk(N)), dim3(256), 0, s, N, (const double*)d, v, h->Dd + (i64)i * N,
                           h->eta + i, (const double*)h->scal, h->flag);
        hipLaunchKernelGGL(k_count, dim3(1), dim3(1), 0, s, h->flag, (const double*)h->scal);
        HIPCHK(h, hipMemcpyAsync(X, v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(h, apply_sop(h, so, s));
        hipLaunchKernelGGL(k_resid2, dim3(nblk(N)), dim3(256), 0, s, N, b, Y, r, X, (const int*)h->flag);
        HIPCHK(h, hipMemcpyAsync(X, r, N * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
    }
    HIPCHK(h, hipGetLastError());
    double hs[5] = {0, 0, 0, 0, 0};
    HIPCHK(h, hipMemcpyAsync(hflag, h->flag, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(hs, h->scal, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (hflag[0] != 0) break;
    batch = std::max(1, check_every);
    const double rr = hs[0], target = hs[4] * hs[3];
    if (tol > 0 && rr_last > 0 && rr > 0 && rr < rr_last && target > 0 && i > i_last) {
      const double rate = std::log(rr / rr_last) / (i - i_last);        // per iteration, < 0
      const double left = std::log(target / rr) / rate;
      if (left >= 0 && left < batch) batch = std::max(1, (int)std::ceil(left) + 1);
    }
    rr_last = rr;
    i_last = i;
  }
  if (hflag[0] == 4) {                   // diverged: back to the iterate with the smallest residual
    HIPCHK(h, hipMemcpyAsync(v, vbest, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
    *n_out = start + hflag[2];
  } else {
    *n_out = start + hflag[1];
  }
  *state_out = hflag[0];
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// C (M x Nc, row-major) = A (M x K, rows contiguous, ld lda) * B^T with B
// (Nc x K, rows contiguous, ld ldb), for short M, Nc and long K: the K range
// is cut into chunks that run as batches of one GEMM stage into partial
// products, summed in chunk order afterwards (deterministic).  Stages are
// appended to `st`; part must hold nch * M * Nc doubles.
// ---------------------------------------------------------------------------
static int long_k_chunks(i64 K) { return (int)std::max<i64>(1, std::min<i64>(64, K / 2048)); }

static void add_long_k(std::vector<Stage>& st, double* C, const double* A, i64 lda, const double* B, i64 ldb, int M,
                       int Nc, i64 K, double* part) {
  const int nch = long_k_chunks(K);
  const i64 kc = K / nch, tail = K - (i64)(nch - 1) * kc;
  Stage g;
  GemmDesc D = desc1(part, Nc, A, lda, 1, B, 1, ldb, M, Nc, (int)kc, 1.0, 0.0, 0);
  D.batch = nch - 1;
  D.c_bs = (i64)M * Nc;
  D.seg[0].a_bs = kc;
  D.seg[0].b_bs = kc;
  if (nch > 1) g.descs.push_back(D);
  g.descs.push_back(desc1(part + (i64)(nch - 1) * M * Nc, Nc, A + (i64)(nch - 1) * kc, lda, 1,
                          B + (i64)(nch - 1) * kc, 1, ldb, M, Nc, (int)tail, 1.0, 0.0, 0));
  st.push_back(g);
  (void)C;
}

// ---------------------------------------------------------------------------
// Float64 re-stabilisation of a block of directions found with the
// low-precision operator (the mixed path).  Directions [i0, i0 + n) of Dd are
// S-conjugated in float64 against the stored ones, which are exact in float64:
//   B = block, SB = S B (float64 operator, the block as nrhs = m right-hand sides);
//   twice: C = eta^-1 o (D^T SB), B -= D C, SB -= (S D) C;
//   P = B^T S B = L L^T (the small projected Cholesky), B <- B L^{-T}, SB <- SB L^{-T},
// so the block's directions are S-orthonormal (eta = 1) in float64 and the
// combined posterior is exact for the space they span.  The weights become
// v = v0 + B (B^T b) (v0: the weights before the block).  Returns GPFVM_E_NOTPD
// if P is not numerically positive definite (nothing stored then).
// ---------------------------------------------------------------------------
static int restabilise_block(gpfvm_handle* h, gpfvm_sop* sm, int i0, int n, const double* v0, Arena& tmp,
                             hipStream_t s) {
  const i64 N = h->N;
  const int m = sm->nrhs;
  double* X = (double*)sm->X;
  double* Y = (double*)sm->Y;
  const int nch = long_k_chunks(N);
  double* Cb = (double*)tmp.alloc((size_t)std::max(i0, 1) * n * sizeof(double));
  double* P = (double*)tmp.alloc((size_t)n * n * sizeof(double));
  double* Pi = (double*)tmp.alloc((size_t)n * n * sizeof(double));
  double* wc = (double*)tmp.alloc((size_t)n * sizeof(double));
  double* part = (double*)tmp.alloc((size_t)nch * std::max(i0, n) * n * sizeof(double));
  if (!Cb || !P || !Pi || !wc || !part) { h->err = "out of device memory (re-stabilisation)"; return GPFVM_E_NOMEM; }
  HIPCHK(h, hipMemcpyAsync(X, h->Dd + (i64)i0 * N, (size_t)n * N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (n < m) HIPCHK(h, launch_fill(X + (i64)n * N, 0.0, (i64)(m - n) * N, s));
  HIPCHK(h, apply_sop(h, sm, s));                                       // Y = S X (float64)
  std::vector<Stage> st;
  if (i0 > 0) {
    // C = D^T SB (i0 x n), then B -= D (C / eta), SB -= (S D) (C / eta)
    Stage c2;
    add_long_k(st, Cb, h->Dd, N, Y, N, i0, n, N, part);                  // partials of D^T SB
    c2.descs.push_back(desc1(X, N, Cb, 1, n, h->Dd, N, 1, n, (int)N, i0, -1.0, 1.0, 0));
    c2.descs.push_back(desc1(Y, N, Cb, 1, n, h->Qd, N, 1, n, (int)N, i0, -1.0, 1.0, 0));
    st.push_back(c2);
  }
  {
    Stage up;
    add_long_k(st, P, X, N, Y, N, n, n, N, part);                         // partials of P = B (S B)^T
    // D_block = L^{-1} B, (S D)_block = L^{-1} SB   (rows of B are the directions)
    up.descs.push_back(desc1(h->Dd + (i64)i0 * N, N, Pi, n, 1, X, N, 1, n, (int)N, n, 1.0, 0.0, 1));
    up.descs.push_back(desc1(h->Qd + (i64)i0 * N, N, Pi, n, 1, Y, N, 1, n, (int)N, n, 1.0, 0.0, 1));
    st.push_back(up);
    Stage wb, vu;
    wb.descs.push_back(desc1(wc, 1, h->Dd + (i64)i0 * N, N, 1, h->bS, 1, 1, n, 1, (int)N, 1.0, 0.0, 0));
    GemmDesc V = desc1(h->v, N, wc, n, 1, h->Dd + (i64)i0 * N, N, 1, 1, (int)N, n, 1.0, 0.0, 0);
    V.X = v0; V.x_rs = N; V.x_cs = 1; V.gamma = 1.0;                    // v = v0 + B (B^T b)
    vu.descs.push_back(V);
    st.push_back(wb);
    st.push_back(vu);
  }
  if (upload_stages(st, tmp, s) != hipSuccess) { h->err = "re-stabilisation: descriptor check/upload failed"; return GPFVM_E_HIP; }
  size_t k = 0;
  if (i0 > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      HIPCHK(h, launch_gemm_stage(F64, st[0], s));
      hipLaunchKernelGGL(k_sum_rowscale, dim3(nblk((i64)i0 * n)), dim3(256), 0, s, nch, i0, n, (const double*)part,
                         (const double*)h->eta, Cb);
      HIPCHK(h, launch_gemm_stage(F64, st[1], s));
    }
    k = 2;
  }
  HIPCHK(h, launch_gemm_stage(F64, st[k], s));                          // P
  hipLaunchKernelGGL(k_sum_rowscale, dim3(nblk((i64)n * n)), dim3(256), 0, s, nch, n, n, (const double*)part,
                     (const double*)nullptr, P);
  {
    std::string e;
    const int rc = cholesky_and_inverse(P, Pi, n, tmp, s, e);
    if (rc == GPFVM_E_NOTPD) { h->err = "re-stabilisation: projected block Gram is not positive definite"; return rc; }
    if (rc) { h->err = e; return rc; }
  }
  HIPCHK(h, launch_gemm_stage(F64, st[k + 1], s));                      // directions and S D
  HIPCHK(h, launch_fill(h->eta + i0, 1.0, n, s));
  HIPCHK(h, launch_gemm_stage(F64, st[k + 2], s));                      // B^T b
  HIPCHK(h, launch_gemm_stage(F64, st[k + 3], s));                      // v
  return GPFVM_OK;
}

// Plain conjugate gradients on the volume system in float64 (Sec. 4.1): x, r
// and p only (no stored directions).  p lives in the operator's input buffer.
static int cg_run(gpfvm_handle* h, const double* b, double* x, int max_iter, double tol, int check_every,
                  hipStream_t s, int* iters_out, int* state_out) {
  const i64 N = h->N;
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, 1, F64, &so);
  if (rc) return rc;
  double* p = (double*)so->X;
  const double* Sp = (const double*)so->Y;
  double* r = h->vec;
  double* dotp = h->aux;
  HIPCHK(h, hipMemsetAsync(h->flag, 0, 16 * sizeof(int), s));
  HIPCHK(h, launch_fill(x, 0.0, N, s));
  HIPCHK(h, hipMemcpyAsync(r, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(p, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, launch_dot(N, b, b, dotp, h->scal + 3, s));
  HIPCHK(h, launch_dot(N, b, b, dotp, h->scal + CG_RR, s));
  {
    const double t2 = tol * tol;
    HIPCHK(h, hipMemcpyAsync(h->scal + 4, &t2, sizeof(double), hipMemcpyHostToDevice, s));
  }
  int hflag[2] = {0, 0};
  double hs[5];
  HIPCHK(h, hipMemcpyAsync(hs, h->scal, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (hs[3] == 0.0) { *iters_out = 0; *state_out = 1; return GPFVM_OK; }
  int it = 0;
  while (it < max_iter) {
    const int end = std::min(max_iter, it + std::max(1, check_every));
    for (; it < end; ++it) {
      const int slot = it & 1;
      HIPCHK(h, apply_sop(h, so, s));                                   // S p
      HIPCHK(h, launch_dot(N, p, Sp, dotp, h->scal + CG_PAP, s));
      hipLaunchKernelGGL(k_cg_step, dim3(nblk(N)), dim3(256), 0, s, N, (const double*)p, Sp, x, r,
                         (const double*)h->scal, slot, h->flag);
      HIPCHK(h, launch_dot(N, r, r, dotp, h->scal + CG_RR + (slot ^ 1), s));
      hipLaunchKernelGGL(k_cg_dir, dim3(nblk(N)), dim3(256), 0, s, N, (const double*)r, p, (const double*)h->scal,
                         slot, h->flag);
    }
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(hflag, h->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (hflag[0] != 0) break;
  }
  *iters_out = hflag[1];
  *state_out = hflag[0];
  return GPFVM_OK;
}

static int rel_res(gpfvm_handle* h, const double* v, double* out, hipStream_t s) {
  const i64 N = h->N;
  double* y = h->vec + 3 * N;
  double* dotp = h->aux;
  int rc = apply_S(h, F64, v, y, s);
  if (rc) return rc;
  HIPCHK(h, launch_axpby(N, 1.0, h->bS, -1.0, y, s));      // y = b - S v
  HIPCHK(h, launch_dot(N, y, y, dotp, h->scal + 8, s));
  HIPCHK(h, launch_dot(N, h->bS, h->bS, dotp, h->scal + 9, s));
  double hv[2];
  HIPCHK(h, hipMemcpyAsync(hv, h->scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  *out = hv[1] > 0 ? std::sqrt(hv[0] / hv[1]) : 0.0;
  return GPFVM_OK;
}

extern "C" int gpfvm_weights(gpfvm_handle* h, double* alpha, void* stream);

static int full_residual(gpfvm_handle* h, double* out, hipStream_t s) {
  // ||y - G alpha|| / ||y|| on the whole system
  const i64 n = h->n;
  Arena tmp;
  tmp.cache = h->arena.cache;
  double* a = (double*)tmp.alloc(n * sizeof(double));
  double* g = (double*)tmp.alloc(n * sizeof(double));
  if (!a || !g) { tmp.release(); h->err = "out of device memory"; return GPFVM_E_NOMEM; }
  int rc = gpfvm_weights(h, a, s);
  if (!rc) rc = gpfvm_matvec(h, 1, a, g, GPFVM_DTYPE_F64, GPFVM_PREC_FP64, s);
  if (!rc) {
    double* dotp = h->aux;
    hipError_t e = launch_axpby(n, 1.0, h->yobs, -1.0, g, s);
    if (e == hipSuccess) e = launch_dot(n, g, g, dotp, h->scal + 10, s);
    if (e == hipSuccess) e = launch_dot(n, h->yobs, h->yobs, dotp, h->scal + 11, s);
    double hv[2] = {0, 1};
    if (e == hipSuccess) e = hipMemcpyAsync(hv, h->scal + 10, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { h->err = hipGetErrorString(e); rc = GPFVM_E_HIP; }
    *out = hv[1] > 0 ? std::sqrt(hv[0] / hv[1]) : 0.0;
  }
  (void)hipStreamSynchronize(s);
  tmp.release();
  return rc;
}

// ---------------------------------------------------------------------------
// Coarse-scheme warm start (appendix "Multigrid preconditioners"): exact
// conditioning on nested coarse volumes before the CG iterations.  Coarse cell
// a is the union of f[0] x ... x f[d-1] fine cells; its observation is the sum
// of theirs (eq. subdomain-partition), i.e. the IterGP action C^T e_a on the
// fine volume system.  The block of Nc such actions is solved exactly: with
// C S C^T = L L^T the directions D0 = C^T L^{-T} are S-orthonormal (eta = 1),
// S D0 = (S C^T) L^{-T}, and the weights start at v0 = D0 D0^T b.
// ---------------------------------------------------------------------------
namespace {

struct CoarseGeom {
  int d;
  int nc[3];   // fine cells per dimension
  int f[3];    // coarsening factors
  int cc[3];   // coarse cells per dimension
};

__device__ __forceinline__ i64 coarse_of(const CoarseGeom& g, i64 i) {
  int idx[3] = {0, 0, 0};
  for (int k = g.d - 1; k >= 0; --k) {
    idx[k] = (int)(i % g.nc[k]);
    i /= g.nc[k];
  }
  i64 a = 0;
  for (int k = 0; k < g.d; ++k) a = a * g.cc[k] + idx[k] / g.f[k];
  return a;
}

// C[a][i] = 1 if fine cell i lies in coarse cell a (Nc x N, row-major)
__global__ void k_coarse_indicator(CoarseGeom g, i64 Nc, i64 N, double* __restrict__ C) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nc * N) return;
  const i64 a = e / N, i = e % N;
  C[e] = coarse_of(g, i) == a ? 1.0 : 0.0;
}

// Gc[a][b] = sum over the fine cells i of coarse cell a of SC[b][i] (fine cells in row-major order)
__global__ void k_coarse_gram(CoarseGeom g, i64 Nc, i64 N, const double* __restrict__ SC, double* __restrict__ Gc) {
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nc * Nc) return;
  const i64 a = e / Nc, b = e % Nc;
  int ac[3] = {0, 0, 0};
  i64 t = a;
  for (int k = g.d - 1; k >= 0; --k) {
    ac[k] = (int)(t % g.cc[k]);
    t /= g.cc[k];
  }
  const int f1 = g.d > 1 ? g.f[1] : 1, f2 = g.d > 2 ? g.f[2] : 1;
  double s = 0.0;
  for (int j0 = 0; j0 < g.f[0]; ++j0)
    for (int j1 = 0; j1 < f1; ++j1)
      for (int j2 = 0; j2 < f2; ++j2) {
        const int i0 = ac[0] * g.f[0] + j0;
        i64 i = i0;
        if (g.d > 1) i = i * g.nc[1] + (ac[1] * g.f[1] + j1);
        if (g.d > 2) i = i * g.nc[2] + (ac[2] * g.f[2] + j2);
        s += SC[b * N + i];
      }
  Gc[e] = s;
}

}  // namespace

// Fills Dd, Qd and eta for the first Nc directions and v with v0; returns Nc through *nc_out.
static int coarse_init(gpfvm_handle* h, const int* factors, hipStream_t s, int* nc_out) {
  const int d = h->d;
  const i64 N = h->N;
  CoarseGeom g{};
  g.d = d;
  i64 Nc = 1;
  for (int k = 0; k < 3; ++k) { g.nc[k] = 1; g.f[k] = 1; g.cc[k] = 1; }
  for (int k = 0; k < d; ++k) {
    g.nc[k] = h->nc[k];
    g.f[k] = factors[k];
    g.cc[k] = h->nc[k] / factors[k];
    Nc *= g.cc[k];
  }
  if (!h->Qd) {
    h->Qd = (double*)h->arena.alloc((size_t)N * h->max_iter * sizeof(double));
    if (!h->Qd) { h->err = "out of device memory (S D store; lower max_iter)"; return GPFVM_E_NOMEM; }
  }
  Arena tmp;
  tmp.cache = h->arena.cache;
  auto fail = [&](int code, const std::string& m) { h->err = m; (void)hipStreamSynchronize(s); tmp.release(); return code; };
  double* C = (double*)tmp.alloc((size_t)Nc * N * sizeof(double));
  double* SC = (double*)tmp.alloc((size_t)Nc * N * sizeof(double));
  double* R = (double*)tmp.alloc((size_t)Nc * N * sizeof(double));
  double* Gc = (double*)tmp.alloc((size_t)Nc * Nc * sizeof(double));
  double* Lic = (double*)tmp.alloc((size_t)Nc * Nc * sizeof(double));
  if (!C || !SC || !R || !Gc || !Lic) return fail(GPFVM_E_NOMEM, "coarse warm start: out of device memory");
  hipLaunchKernelGGL(k_coarse_indicator, dim3((unsigned)((Nc * N + 255) / 256)), dim3(256), 0, s, g, Nc, N, C);
  // S C^T, a batch of right-hand sides at a time (rows of C are the rhs, N apart)
  const int B = (int)std::min<i64>(Nc, 64);
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, B, F64, &so);
  if (rc) { (void)hipStreamSynchronize(s); tmp.release(); return rc; }
  for (i64 j0 = 0; j0 < Nc; j0 += B) {
    const i64 nr = std::min<i64>(B, Nc - j0);
    if (hipMemcpyAsync(so->X, C + j0 * N, (size_t)nr * N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(GPFVM_E_HIP, "coarse warm start: copy failed");
    if (nr < B && launch_fill((double*)so->X + nr * N, 0.0, (B - nr) * N, s) != hipSuccess)
      return fail(GPFVM_E_HIP, "coarse warm start: fill failed");
    if (apply_sop(h, so, s) != hipSuccess) return fail(GPFVM_E_HIP, "coarse warm start: operator failed");
    if (hipMemcpyAsync(SC + j0 * N, so->Y, (size_t)nr * N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(GPFVM_E_HIP, "coarse warm start: copy failed");
  }
  hipLaunchKernelGGL(k_coarse_gram, dim3((unsigned)((Nc * Nc + 255) / 256)), dim3(256), 0, s, g, Nc, N,
                     (const double*)SC, Gc);
  rc = cholesky_and_inverse(Gc, Lic, (int)Nc, tmp, s, h->err);
  if (rc) {
    if (rc == GPFVM_E_NOTPD) h->err = "coarse warm start: C S C^T is not positive definite";
    (void)hipStreamSynchronize(s);
    tmp.release();
    return rc;
  }
  // Dd[0:Nc] = L^{-1} C and Qd[0:Nc] = L^{-1} (S C^T)^T, each as T = Linv B ; R = B - L T ; T += Linv R
  const int n = (int)Nc;
  std::vector<Stage> st(6);
  double* outs[2] = {h->Dd, h->Qd};
  const double* ins[2] = {C, SC};
  for (int q = 0; q < 2; ++q) {
    st[3 * q].descs.push_back(desc1(outs[q], N, Lic, n, 1, ins[q], N, 1, n, (int)N, n, 1.0, 0.0, 1));
    GemmDesc D = desc1(R, N, Gc, n, 1, outs[q], N, 1, n, (int)N, n, -1.0, 0.0, 1);
    D.X = ins[q]; D.x_rs = N; D.x_cs = 1; D.gamma = 1.0;
    st[3 * q + 1].descs.push_back(D);
    st[3 * q + 2].descs.push_back(desc1(outs[q], N, Lic, n, 1, R, N, 1, n, (int)N, n, 1.0, 1.0, 1));
  }
  // A second orthonormalisation of the block in the S inner product (Cholesky QR twice):
  // with C S C^T of condition ~1e9 (4 x 4 fine cells per coarse cell on advection-diffusion
  // 128^2) the directions above are S-orthonormal only to ~1e-7, while the CG phase takes
  // eta = 1 for them.  P = D0 (S D0)^T = L2 L2^T, D0 <- L2^{-1} D0, S D0 <- L2^{-1} S D0
  // brings the block to S-orthonormality at rounding level (there the smallest residual
  // of the CG phase drops from 1.9e-8 to 9e-9).  It spans the same space, so the
  // conditioning it represents is unchanged.  Gc, Lic, C and SC are free for reuse here.
  const int nch = long_k_chunks(N);
  double* part = (double*)tmp.alloc((size_t)nch * n * n * sizeof(double));
  if (!part) return fail(GPFVM_E_NOMEM, "coarse warm start: out of device memory");
  std::vector<Stage> st2;
  add_long_k(st2, Gc, h->Dd, N, h->Qd, N, n, n, N, part);              // partials of P
  {
    Stage up;
    up.descs.push_back(desc1(h->Dd, N, Lic, n, 1, C, N, 1, n, (int)N, n, 1.0, 0.0, 1));
    up.descs.push_back(desc1(h->Qd, N, Lic, n, 1, SC, N, 1, n, (int)N, n, 1.0, 0.0, 1));
    st2.push_back(up);
  }
  if (upload_stages(st, tmp, s) != hipSuccess || upload_stages(st2, tmp, s) != hipSuccess)
    return fail(GPFVM_E_HIP, "coarse warm start: upload failed");
  if (run_stages(st, s) != hipSuccess) return fail(GPFVM_E_HIP, "coarse warm start: gemm failed");
  if (launch_gemm_stage(F64, st2[0], s) != hipSuccess) return fail(GPFVM_E_HIP, "coarse warm start: gemm failed");
  hipLaunchKernelGGL(k_sum_rowscale, dim3(nblk((i64)n * n)), dim3(256), 0, s, nch, n, n, (const double*)part,
                     (const double*)nullptr, Gc);
  rc = cholesky_and_inverse(Gc, Lic, n, tmp, s, h->err);
  if (rc) {
    if (rc == GPFVM_E_NOTPD) h->err = "coarse warm start: the projected coarse Gram is not positive definite";
    (void)hipStreamSynchronize(s);
    tmp.release();
    return rc;
  }
  if (hipMemcpyAsync(C, h->Dd, (size_t)n * N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(SC, h->Qd, (size_t)n * N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(GPFVM_E_HIP, "coarse warm start: copy failed");
  if (launch_gemm_stage(F64, st2[1], s) != hipSuccess) return fail(GPFVM_E_HIP, "coarse warm start: gemm failed");
  // eta = 1 ; v = D0 (D0^T b): the column update gives -D0 c from base 0, negated after
  double* coef = h->aux + 1024;
  if (launch_fill(h->eta, 1.0, Nc, s) != hipSuccess || launch_fill(h->v, 0.0, N, s) != hipSuccess ||
      launch_rows_dot(n, N, h->Dd, h->bS, coef, s) != hipSuccess ||
      launch_cols_update(n, N, h->Dd, coef, rows_dot_chunks(n, N), h->eta, h->v, h->v, nullptr, nullptr, nullptr,
                         nullptr, s) != hipSuccess ||
      launch_axpby(N, 0.0, h->v, -1.0, h->v, s) != hipSuccess)
    return fail(GPFVM_E_HIP, "coarse warm start: launch failed");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(GPFVM_E_HIP, "coarse warm start: kernel failed");
  tmp.release();
  *nc_out = n;
  return GPFVM_OK;
}

extern "C" int gpfvm_solve(gpfvm_handle* h, const gpfvm_solve_opts* o, gpfvm_solve_info* info, void* stream) {
  if (!h) return GPFVM_E_INVALID;
  gpfvm_solve_opts def;
  gpfvm_default_solve_opts(&def);
  if (!o) o = &def;
  if (o->prec != GPFVM_PREC_FP64 && o->prec != GPFVM_PREC_MIXED) { h->err = "solve: bad prec"; return GPFVM_E_INVALID; }
  if (o->method != GPFVM_METHOD_ITERGP && o->method != GPFVM_METHOD_CG) { h->err = "solve: bad method"; return GPFVM_E_INVALID; }
  if (o->prec == GPFVM_PREC_MIXED && h->multi) {
    h->err = "solve: the mixed path takes single-output problems";
    return GPFVM_E_INVALID;
  }
  if (o->prec == GPFVM_PREC_MIXED && o->tile != h->tile) {
    h->err = "solve: the mixed path's tile format must be the one given at assemble";
    return GPFVM_E_INVALID;
  }
  if (o->max_iter < 0 || !(o->tol >= 0) || o->check_every < 1 || o->max_outer < 1 || o->block < 1 ||
      o->block > GPFVM_MAX_BLOCK || o->reorth_passes < 1 || o->reorth_passes > 2 || o->replace_every < 1) {
    h->err = "solve: bad options";
    return GPFVM_E_INVALID;
  }
  if (o->prec == GPFVM_PREC_MIXED && o->reorth_passes != 2) {
    h->err = "solve: the mixed path needs reorth_passes = 2";
    return GPFVM_E_INVALID;
  }
  if (o->method == GPFVM_METHOD_CG && (o->prec != GPFVM_PREC_FP64 || o->resume)) {
    h->err = "solve: method CG is float64 and does not resume";
    return GPFVM_E_INVALID;
  }
  if (o->resume && (!h->solved || h->cg_only)) { h->err = "solve: nothing to resume"; return GPFVM_E_STATE; }
  // coarse warm start: factors >= 1 dividing the cell counts; all 1 = off
  i64 n_coarse = 1;
  bool coarse = false;
  for (int k = 0; k < h->d; ++k) {
    const int f = o->coarsen[k];
    if (f < 1 || h->nc[k] % f != 0) { h->err = "solve: coarsening factors must divide the cell counts"; return GPFVM_E_INVALID; }
    n_coarse *= h->nc[k] / f;
    coarse |= (f > 1);
  }
  if (coarse && h->multi) {
    h->err = "solve: the coarse warm start takes single-output problems";
    return GPFVM_E_INVALID;
  }
  if (coarse) {
    if (o->resume || o->prec != GPFVM_PREC_FP64 || o->reorth_passes != 2 || o->method != GPFVM_METHOD_ITERGP) {
      h->err = "solve: the coarse warm start needs a fresh float64 solve with reorth_passes = 2";
      return GPFVM_E_INVALID;
    }
    if (n_coarse >= h->max_iter || n_coarse > GPFVM_MAX_COARSE) {
      h->err = "solve: too many coarse cells for the direction capacity (assemble max_iter) or the limit";
      return GPFVM_E_INVALID;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  int rc = ensure_state(h, s);
  if (rc) return rc;
  const i64 N = h->N;
  int n_dirs_coarse = 0;
  if (!o->resume) {
    HIPCHK(h, launch_fill(h->v, 0.0, N, s));
    h->iters = 0;
    h->sd_exact = true;
    h->solved = false;
    if (coarse) {
      rc = coarse_init(h, o->coarsen, s, &n_dirs_coarse);
      if (rc) return rc;
      h->iters = n_dirs_coarse;
    }
  }
  // S D holds float64 S D after float64 two-pass iterations and after the mixed
  // path's re-stabilised blocks, not after one-pass iterations
  if (o->reorth_passes != 2) h->sd_exact = false;
  int state = 0, outer = 0;
  h->cg_only = false;
  int cg_iters = 0;
  if (o->method == GPFVM_METHOD_CG) {
    rc = cg_run(h, h->bS, h->v, o->max_iter, o->tol, o->check_every, s, &cg_iters, &state);
    if (rc) return rc;
    h->iters = 0;
    h->cg_only = true;
    h->sd_exact = false;
  } else if (o->prec == GPFVM_PREC_FP64) {
    int nd = h->iters;
    const int start0 = h->iters;
    rc = itergp_run(h, F64, h->bS, h->v, h->iters, o->max_iter, o->tol, o->check_every, o->reorth_passes,
                    o->replace_every, s, &nd, &state);
    if (rc) return rc;
    h->iters = nd;
    // The stopping test reads the recursive residual.  Where the explicit residual is still
    // above the tolerance and the budget allows, continue from it (the loop starts from
    // r = b - S v, a residual replacement), at most twice.
    for (int again = 0; again < 2 && state == 1 && o->tol > 0; ++again) {
      const int left = o->max_iter - (h->iters - start0);
      if (left <= 0 || h->iters >= h->max_iter) break;
      double r0 = 0;
      rc = rel_res(h, h->v, &r0, s);
      if (rc) return rc;
      if (r0 <= o->tol) break;
      rc = itergp_run(h, F64, h->bS, h->v, h->iters, left, o->tol, o->check_every, o->reorth_passes,
                      o->replace_every, s, &nd, &state);
      if (rc) return rc;
      h->iters = nd;
    }
  } else {
    // Mixed precision: blocks of up to `block` IterGP iterations with the
    // low-precision operator (its directions projected twice against every
    // stored direction, in float64), each started from the float64 residual
    // b - S v and followed by the float64 re-stabilisation of its directions
    // (restabilise_block: float64 S D, the small projected Cholesky, weights
    // v = C b).  The float64 residual at the start of the next block is the
    // refinement step.  If a block cannot add a direction (eta <= 0 at once,
    // or a block Gram that is not positive definite) the solve continues with
    // the float64 operator.
    gpfvm_sop* sm = nullptr;
    rc = get_sop(h, o->block, F64, &sm);
    if (rc) return rc;
    if (!h->Qd) {
      h->Qd = (double*)h->arena.alloc((size_t)N * h->max_iter * sizeof(double));
      if (!h->Qd) { h->err = "out of device memory (S D store; lower max_iter)"; return GPFVM_E_NOMEM; }
    }
    Arena tmp;
    tmp.cache = h->arena.cache;
    double* vsave = (double*)tmp.alloc((size_t)N * sizeof(double));
    if (!vsave) { tmp.release(); h->err = "out of device memory (mixed path)"; return GPFVM_E_NOMEM; }
    const int start0 = h->iters, end = std::min(h->max_iter, start0 + o->max_iter);
    bool fall_back = false;
    for (outer = 0; outer < o->max_outer && h->iters < end; ++outer) {
      HIPCHK(h, hipMemcpyAsync(vsave, h->v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
      int nd = h->iters;
      rc = itergp_run(h, F32, h->bS, h->v, h->iters, std::min(o->block, end - h->iters), o->tol, o->check_every, 2,
                      1 << 30, s, &nd, &state, nullptr, true);
      if (rc) { tmp.release(); return rc; }
      const int nnew = nd - h->iters;
      if (nnew == 0) {
        HIPCHK(h, hipMemcpyAsync(h->v, vsave, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        fall_back = (state != 1);               // converged at the block's float64 residual, or stuck
        break;
      }
      rc = restabilise_block(h, sm, h->iters, nnew, vsave, tmp, s);
      if (rc == GPFVM_E_NOTPD) {               // drop the block
        HIPCHK(h, hipMemcpyAsync(h->v, vsave, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        fall_back = true;
        break;
      }
      if (rc) { tmp.release(); return rc; }
      h->iters = nd;
      state = 0;
    }
    tmp.release();
    if (fall_back && h->iters < end) {
      int nd = h->iters;
      rc = itergp_run(h, F64, h->bS, h->v, h->iters, end - h->iters, o->tol, o->check_every, 2, o->replace_every, s,
                      &nd, &state);
      if (rc) return rc;
      h->iters = nd;
    }
    double res = 0;
    rc = rel_res(h, h->v, &res, s);
    if (rc) return rc;
    state = (o->tol > 0 && res <= o->tol) ? 1 : (state == 2 ? 2 : 3);
  }
  h->solved = true;
  double rs = 0, rf = 0;
  rc = rel_res(h, h->v, &rs, s);
  if (rc) return rc;
  rc = full_residual(h, &rf, s);
  if (rc) return rc;
  if (info) {
    info->iters = h->cg_only ? cg_iters : h->iters;
    info->outer = outer;
    info->rel_res = rs;
    info->rel_res_full = rf;
    info->status = GPFVM_OK;
    info->coarse = n_dirs_coarse;
  }
  int status = GPFVM_OK;
  if (state == 2) status = GPFVM_E_NOTPD;
  else if (o->tol > 0 && rs > o->tol) status = GPFVM_E_NOCONV;
  if (info) info->status = status;
  if (status == GPFVM_E_NOTPD) h->err = "IterGP breakdown: eta <= 0 (state kept up to the last good direction)";
  if (status == GPFVM_E_NOCONV)
    h->err = state == 4 ? "the residual grew 1000-fold above its smallest value (the tolerance is below the "
                          "attainable accuracy); state rolled back to the iterate with the smallest residual"
                        : "iteration budget exhausted above the tolerance";
  return status;
}

// ---------------------------------------------------------------------------
// Targeted uncertainty reduction (appendix "Targeted uncertainty reduction"):
// `iters` further IterGP iterations after a solve whose actions are the
// residuals of b_i = K_S(X~) beta_i with respect to the current inverse
// approximation C = D diag(1/eta) D^T,  s_i = b_i - S C b_i = b_i - (S D)(eta^-1 o D^T b_i),
// using the stored images S D (no extra operator application).  K_S(X~) is the
// volume-target cross-covariance under the IC/BC-conditioned prior,
// L_V k(X~) - G_pb G_bb^{-1} L_b k(X~); X~ is a tensor grid and beta_i the i-th
// row of `weights` (host, iters x prod(n)).  The representer weights take the
// usual IterGP step with the data residual; the directions are appended.
// ---------------------------------------------------------------------------
extern "C" int gpfvm_refine_variance(gpfvm_handle* h, int dim, const int* n, const double* const* axis, int iters,
                                     const double* weights, gpfvm_solve_info* info, void* stream) {
  if (!h) return GPFVM_E_INVALID;
  if (h->multi) { h->err = "refine_variance: targeted reduction takes single-output problems"; return GPFVM_E_INVALID; }
  if (dim != h->d || !n || !axis) { h->err = "refine_variance: bad target grid"; return GPFVM_E_INVALID; }
  i64 M = 1;
  for (int i = 0; i < dim; ++i) {
    if (n[i] < 1 || !axis[i]) { h->err = "refine_variance: bad target axis"; return GPFVM_E_INVALID; }
    for (int j = 0; j < n[i]; ++j)
      if (!std::isfinite(axis[i][j])) { h->err = "refine_variance: non-finite target"; return GPFVM_E_INVALID; }
    M *= n[i];
  }
  if (iters < 1 || !weights) { h->err = "refine_variance: bad iteration count or weights"; return GPFVM_E_INVALID; }
  for (i64 k = 0; k < (i64)iters * M; ++k)
    if (!std::isfinite(weights[k])) { h->err = "refine_variance: non-finite weights"; return GPFVM_E_INVALID; }
  if (!h->solved) { h->err = "refine_variance: no solve yet"; return GPFVM_E_STATE; }
  if (!h->sd_exact) {
    h->err = "refine_variance: needs a float64 solve with two projection passes (the stored S D images)";
    return GPFVM_E_STATE;
  }
  if (h->iters + iters > h->max_iter) {
    h->err = "refine_variance: direction capacity (assemble max_iter) exceeded";
    return GPFVM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  int rc = ensure_state(h, s);
  if (rc) return rc;
  gpfvm_sop* so = nullptr;
  rc = get_sop(h, 1, F64, &so);
  if (rc) return rc;
  const int d = h->d;
  const i64 N = h->N;
  Arena tmp;
  tmp.cache = h->arena.cache;
  auto fail = [&](int code, const std::string& m) { h->err = m; (void)hipStreamSynchronize(s); tmp.release(); return code; };
  double* gax[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < d; ++i) {
    gax[i] = (double*)tmp.alloc(n[i] * sizeof(double));
    if (!gax[i]) return fail(GPFVM_E_NOMEM, "refine_variance: out of device memory");
    if (hipMemcpyAsync(gax[i], axis[i], n[i] * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(GPFVM_E_HIP, "refine_variance: copy failed");
  }
  double* wts = (double*)tmp.alloc((size_t)iters * M * sizeof(double));
  double* beta = (double*)tmp.alloc((size_t)M * sizeof(double));
  if (!wts || !beta) return fail(GPFVM_E_NOMEM, "refine_variance: out of device memory");
  if (hipMemcpyAsync(wts, weights, (size_t)iters * M * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(GPFVM_E_HIP, "refine_variance: copy failed");
  // L_V k(X~): cells <- targets, the adjoint of the posterior's grid operator
  KronOp pt;
  pt.d = d;
  for (int i = 0; i < d; ++i) { pt.in_shape[i] = n[i]; pt.out_shape[i] = h->nc[i]; }
  pt.in_len = M;
  for (size_t t = 0; t < h->pterms.size(); ++t) {
    KronTerm k{};
    for (int i = 0; i < d; ++i) {
      double* Q = (double*)tmp.alloc((size_t)n[i] * h->nc[i] * sizeof(double));
      if (!Q) return fail(GPFVM_E_NOMEM, "refine_variance: out of device memory");
      if (launch_factor(1, h->kq[i], 0, h->pterms[t].alpha[i], n[i], gax[i], h->nc[i], h->edges[i], h->ell[i], 1.0, Q,
                        h->nc[i], s) != hipSuccess)
        return fail(GPFVM_E_HIP, "refine_variance: factor launch failed");
      k.M[i] = Q;
      k.ld[i] = h->nc[i];
      k.trans[i] = 1;
    }
    k.alpha = h->sf2 * h->pterms[t].coef;
    k.lscale = h->pterms[t].cellwise;
    pt.terms.push_back(k);
  }
  // L_b k(X~): points of each group <- targets
  std::vector<KronOp> bt;
  for (size_t g = 0; g < h->groups.size(); ++g) {
    const Group& Gr = h->groups[g];
    KronOp o;
    o.d = d;
    for (int i = 0; i < d; ++i) { o.in_shape[i] = n[i]; o.out_shape[i] = Gr.n[i]; }
    o.in_len = M;
    o.out_off = Gr.offset;
    KronTerm k{};
    for (int i = 0; i < d; ++i) {
      double* ga = (double*)tmp.alloc(Gr.n[i] * sizeof(double));
      double* P = (double*)tmp.alloc((size_t)Gr.n[i] * n[i] * sizeof(double));
      if (!ga || !P) return fail(GPFVM_E_NOMEM, "refine_variance: out of device memory");
      if (hipMemcpyAsync(ga, Gr.axis[i].data(), Gr.n[i] * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(GPFVM_E_HIP, "refine_variance: copy failed");
      // P[b][x] = d^beta_b k(x_b, x)
      if (launch_factor(2, h->kq[i], Gr.deriv[i], 0, Gr.n[i], ga, n[i], gax[i], h->ell[i], 1.0, P, n[i], s) !=
          hipSuccess)
        return fail(GPFVM_E_HIP, "refine_variance: factor launch failed");
      k.M[i] = P;
      k.ld[i] = n[i];
    }
    k.alpha = h->sf2;
    o.terms.push_back(k);
    bt.push_back(o);
  }
  Plan ppt, pbt;
  {
    std::vector<KronOp> ops{pt};
    rc = compile_kron_list(ops, F64, 1, beta, M, so->Y, N, h->cellc, h->cellc, 0.0, nullptr, 0, 1, tmp, s, ppt, h->err);
    if (rc) { tmp.release(); return rc; }
    if (h->nb > 0) {
      rc = compile_kron_list(bt, F64, 1, beta, M, so->U, h->nb, nullptr, nullptr, 0.0, nullptr, 0, 0, tmp, s, pbt,
                             h->err);
      if (rc) { tmp.release(); return rc; }
    }
  }
  double* X = (double*)so->X;
  double* Y = (double*)so->Y;
  double* coef = h->aux + 1024;
  const int start = h->iters;
  // X = b_i - (S D) (eta^-1 o D^T b_i),  b_i = K_S(X~) beta_i (built in Y)
  std::function<int(int)> action = [&](int i) -> int {
    HIPCHK(h, hipMemcpyAsync(beta, wts + (i64)(i - start) * M, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, run_plan(ppt, s));
    if (h->nb > 0) {
      HIPCHK(h, run_plan(pbt, s));
      HIPCHK(h, apply_ginv(h, so, s));
      HIPCHK(h, run_plan(so->pb, s));                       // Y -= G_pb G_bb^{-1} L_b k(X~) beta
    }
    if (i > 0) {
      HIPCHK(h, launch_rows_dot(i, N, h->Dd, Y, coef, s));
      HIPCHK(h, launch_cols_update(i, N, h->Qd, coef, rows_dot_chunks(i, N), h->eta, Y, X, nullptr, nullptr, nullptr,
                                   nullptr, s));
    } else {
      HIPCHK(h, hipMemcpyAsync(X, Y, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    return GPFVM_OK;
  };
  int nd = start, state = 0;
  rc = itergp_run(h, F64, h->bS, h->v, start, iters, 0.0, 16, 2, 25, s, &nd, &state, &action);
  if (rc) { (void)hipStreamSynchronize(s); tmp.release(); return rc; }
  h->iters = nd;
  if (hipStreamSynchronize(s) != hipSuccess) return fail(GPFVM_E_HIP, "refine_variance: kernel failed");
  tmp.release();
  double rs = 0, rf = 0;
  rc = rel_res(h, h->v, &rs, s);
  if (rc) return rc;
  rc = full_residual(h, &rf, s);
  if (rc) return rc;
  const int status = (state == 2) ? GPFVM_E_NOTPD : GPFVM_OK;
  if (info) {
    info->iters = h->iters;
    info->outer = 0;
    info->rel_res = rs;
    info->rel_res_full = rf;
    info->status = status;
    info->coarse = 0;
  }
  if (status == GPFVM_E_NOTPD) h->err = "IterGP breakdown: eta <= 0 (state kept up to the last good direction)";
  return status;
}

extern "C" int gpfvm_weights(gpfvm_handle* h, double* alpha, void* stream) {
  if (!h || !alpha) return GPFVM_E_INVALID;
  if (!h->solved) { h->err = "weights: no solve yet"; return GPFVM_E_STATE; }
  hipStream_t s = (hipStream_t)stream;
  const i64 N = h->N;
  HIPCHK(h, hipMemcpyAsync(alpha + h->nb, h->v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h->nb > 0) {
    // alpha_b = G_bb^{-1} (y_b - G_bp v)
    gpfvm_sop* so = nullptr;
    int rc = get_sop(h, 1, F64, &so);
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(so->X, h->v, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, run_plan(so->bp, s));
    HIPCHK(h, launch_axpby(h->nb, 1.0, h->yobs, -1.0, (double*)so->U, s));
    HIPCHK(h, apply_ginv(h, so, s));     // the one-vector form (one workgroup or row-streaming)
    HIPCHK(h, hipMemcpyAsync(alpha, so->W, h->nb * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return GPFVM_OK;
}

// ---------------------------------------------------------------------------
// posterior on a tensor grid
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Point part of the posterior variance, ||L^{-1} k_b(x)||^2, group by group
// (Sec. 2.1 eq. lin-cond-cov with the point groups' tensor grids, Sec. 2.2).
// A group's points form a tensor grid, so its rows of k_b(x) are
// sf2 prod_i P_{g,i}[p_i][x_i].  In a dimension where the group has a single
// point (initial data at one time, an edge at one position) that factor is a
// scalar w per grid coordinate, so
//   k_b(x) = sum_g w_g(x) E_g B_g[:, a_g(x)],
// with B_g the group's points x free grid coordinates factor, a_g(x) the grid
// point's free coordinates and E_g placing the group's rows.  Then
//   L^{-1} k_b(x) = sum_g w_g(x) U_g[:, a_g(x)],   U_g = L^{-1} E_g B_g,
// with one column per free grid coordinate of the group (its rows above the
// group's offset are zero, L^{-1} being lower-triangular).  The vector is
// formed row by row and squared: expanding the norm into the groups' pairwise
// inner products instead loses digits to cancellation (the solved columns of
// two groups on the same points, u and u_t at t = 0, are large and nearly
// opposite; on the wave problem the variance moved 1.8e-7 from the oracle's).
// On the wave problem this solves 36 864 columns instead of 131 072 and touches
// only each group's rows of L^{-1}.
// ---------------------------------------------------------------------------
constexpr int GV_MAXG = 12;                  // (group, component) pairs handled by the grouped form
struct GVGroupDev {
  i64 off, C;                                // row offset, columns (free grid coordinates)
  i64 cs[3];                                 // column stride of each free grid coordinate (0 if pinned)
  const double* U;                           // (nb - off) x C, row-major
  const double* W[3];                        // pinned dimensions: the factor row (1 x gdim), else null
};
struct GVMeta {
  int d, ngroup;
  int gdim[3];
  GVGroupDev grp[GV_MAXG];
};
struct GVFactor {                            // one group's B_g^T (free grid coordinates x points)
  int d;
  int pn[3];                                 // the group's points per dimension
  int ext[3];                                // grid extent per dimension
  int isfree[3];
  const double* P[3];                        // n_{g,i} x gdim_i
};

// Bt[a][p] = coef prod_{i free} P_i[p_i][a_i]  (a over the free grid coordinates, p over the points)
__global__ void k_gv_bt(GVFactor F, double coef, i64 C, i64 np, double* __restrict__ Bt) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= C * np) return;
  const i64 a = idx / np, p = idx % np;
  int pi[3] = {0, 0, 0}, ai[3] = {0, 0, 0};
  i64 r = p;
  for (int i = F.d - 1; i >= 0; --i) { pi[i] = (int)(r % F.pn[i]); r /= F.pn[i]; }
  r = a;
  for (int i = F.d - 1; i >= 0; --i)
    if (F.isfree[i]) { ai[i] = (int)(r % F.ext[i]); r /= F.ext[i]; }
  double v = coef;
  for (int i = 0; i < F.d; ++i)
    if (F.isfree[i]) v *= F.P[i][(i64)pi[i] * F.ext[i] + ai[i]];
  Bt[idx] = v;
}

// red[x] += sum_r (sum_{g: off_g <= r} w_g(x) U_g[r - off_g][a_g(x)])^2, one thread per grid
// point, rows in order.  Neighbouring grid points differ in the last coordinate, so a
// wavefront's loads of a row of U_g are contiguous or one address.
constexpr int GV_U = 4;
template <int NG>
__global__ __launch_bounds__(256) void k_gv_direct(const GVMeta* __restrict__ meta, i64 M, i64 nb,
                                                   double* __restrict__ red) {
  const GVMeta& V = *meta;
  const i64 x = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= M) return;
  int c[3] = {0, 0, 0};
  i64 rr = x;
  for (int i = V.d - 1; i >= 0; --i) { c[i] = (int)(rr % V.gdim[i]); rr /= V.gdim[i]; }
  double w[NG];
  const double* p[NG];
  i64 C[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const GVGroupDev& G = V.grp[g];
    double wv = 1.0;
    i64 a = 0;
    for (int i = 0; i < V.d; ++i) {
      if (G.W[i]) wv *= G.W[i][c[i]];
      a += (i64)c[i] * G.cs[i];
    }
    w[g] = wv;
    p[g] = G.U + a;                          // row 0 of the group, this point's column
    C[g] = G.C;
  }
  double acc = 0.0;
#pragma unroll
  for (int g1 = 0; g1 < NG; ++g1) {          // rows [off_g1, off_g1+1): groups 0..g1 contribute
    const i64 rlo = V.grp[g1].off, rhi = g1 + 1 < NG ? V.grp[g1 + 1].off : nb;
    i64 r = rlo;
    // four rows at a time: their loads are issued together, then added in the same order
    for (; r + GV_U <= rhi; r += GV_U) {
      double v[GV_U][NG];
#pragma unroll
      for (int u = 0; u < GV_U; ++u)
#pragma unroll
        for (int g = 0; g <= g1; ++g) v[u][g] = p[g][(r + u - V.grp[g].off) * C[g]];
#pragma unroll
      for (int u = 0; u < GV_U; ++u) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g <= g1; ++g) t = fma(w[g], v[u][g], t);
        acc = fma(t, t, acc);
      }
    }
    for (; r < rhi; ++r) {
      double t = 0.0;
#pragma unroll
      for (int g = 0; g <= g1; ++g) t = fma(w[g], p[g][(r - V.grp[g].off) * C[g]], t);
      acc = fma(t, t, acc);
    }
  }
  red[x] += acc;
}

// The grouped point variance into red.  Every (group, component) pair on the output is
// one term of k_b(x) (two components of a group share its rows; their offsets tie, so
// the first one's band of rows is empty and the second's covers both).  Returns 1 when
// it does not apply (more than GV_MAXG pairs, products not clearly cheaper than the
// chunked L^{-1} K_b, or buffers beyond three of its chunk buffers); else a GPFVM code.
static int grouped_point_var(gpfvm_handle* h, const PGMeta& pg, const int* n, i64 M, double* red, Arena& tmp,
                             hipStream_t s) {
  const int d = h->d;
  const i64 nb = h->nb;
  struct Grp { int g, c; double coef; i64 off, np, K, C; int isfree[3]; i64 cs[3]; int nfree; double* Bt; double* U; };
  std::vector<Grp> gr;
  for (int g = 0; g < (int)h->groups.size(); ++g)
    for (int c = 0; c < pg.gcomp[g]; ++c)
      if (pg.pc[g][c] != 0.0) gr.push_back(Grp{g, c, pg.pc[g][c]});
  const int G = (int)gr.size();
  if (G < 1 || G > GV_MAXG) return 1;
  double work = 0, words = 0;
  for (Grp& q : gr) {
    const Group& H = h->groups[q.g];
    q.off = H.offset;
    q.np = 1;
    q.C = 1;
    for (int i = 0; i < 3; ++i) { q.isfree[i] = 0; q.cs[i] = 0; }
    for (int i = 0; i < d; ++i) {
      q.np *= H.n[i];
      q.isfree[i] = H.n[i] > 1;
    }
    for (int i = d - 1; i >= 0; --i) {
      q.cs[i] = q.isfree[i] ? q.C : 0;
      if (q.isfree[i]) q.C *= n[i];
    }
    q.K = nb - q.off;
    q.nfree = 0;
    int fd[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i)
      if (q.isfree[i]) fd[q.nfree++] = i;
    if (q.nfree == 2) {
      // U = X_sub B_g^T as two mode products (B_g^T is the Kronecker product of the free
      // dimensions' point factors): the cheaper order's flops and its intermediate
      const double pa = H.n[fd[0]], pb = H.n[fd[1]], ga = n[fd[0]], gb = n[fd[1]];
      const double w1 = pa * pb * gb + pa * gb * ga, w2 = pa * pb * ga + ga * pb * gb;
      work += (double)q.K * std::min(w1, w2);
      words += (double)q.C * q.K + (double)q.K * std::max(pa * gb, ga * pb);
    } else {
      work += (double)q.K * q.np * q.C;
      words += (double)q.C * q.K + (double)q.C * q.np;
    }
  }
  if (work > 0.25 * (double)nb * nb * M) return 1;
  if (words > 4.0 * nb * posterior_chunk(nb, M)) return 1;     // within the posterior's memory estimate
  for (Grp& q : gr) {
    q.U = (double*)tmp.alloc((size_t)(q.C * q.K) * sizeof(double));
    if (!q.U) { h->err = "posterior: out of device memory"; return GPFVM_E_NOMEM; }
    if (q.nfree == 2) {
      // U (K x C) = X_sub (K x np) B_g^T by the Kronecker plan: the K rows of
      // X_sub = L^{-1}[off:, off:off+np] are its right-hand sides (stride n_b), each a
      // tensor over the group's two free dimensions mapped to the grid's
      KronOp op;
      op.d = 2;
      KronTerm t{};
      int k = 0;
      for (int i = 0; i < d; ++i) {
        if (!q.isfree[i]) continue;
        op.in_shape[k] = h->groups[q.g].n[i];
        op.out_shape[k] = n[i];
        t.M[k] = pg.P[q.g][q.c][i];       // n_{g,i} x grid_i, used transposed
        t.ld[k] = n[i];
        t.trans[k] = 1;
        ++k;
      }
      op.in_len = q.np;
      t.alpha = q.coef;
      op.terms.push_back(t);
      std::vector<KronOp> ops{op};
      Plan pl;
      int rc = compile_kron_list(ops, F64, (int)q.K, h->Linv + q.off * nb + q.off, nb, q.U, q.C, nullptr, nullptr, 0.0,
                                 nullptr, 0, 1, tmp, s, pl, h->err);
      if (rc) return rc;
      if (run_plan(pl, s) != hipSuccess) { h->err = "posterior: group product failed"; return GPFVM_E_HIP; }
      continue;
    }
    q.Bt = (double*)tmp.alloc((size_t)(q.C * q.np) * sizeof(double));
    if (!q.Bt) { h->err = "posterior: out of device memory"; return GPFVM_E_NOMEM; }
    GVFactor F{};
    F.d = d;
    for (int i = 0; i < 3; ++i) { F.pn[i] = 1; F.ext[i] = 1; F.isfree[i] = 0; F.P[i] = nullptr; }
    for (int i = 0; i < d; ++i) {
      F.pn[i] = h->groups[q.g].n[i];
      F.ext[i] = n[i];
      F.isfree[i] = q.isfree[i];
      F.P[i] = pg.P[q.g][q.c][i];
    }
    hipLaunchKernelGGL(k_gv_bt, dim3(nblk(q.C * q.np)), dim3(256), 0, s, F, q.coef, q.C, q.np, q.Bt);
    // U (K x C) = X_sub (K x np) Bt^T, X_sub = L^{-1}[off:, off:off+np]
    if (gemm_rows_abt((int)q.K, (int)q.C, (int)q.np, h->Linv + q.off * nb + q.off, (int)nb, q.Bt, (int)q.np, q.U,
                      (int)q.C, s) != hipSuccess) {
      h->err = "posterior: group product failed";
      return GPFVM_E_HIP;
    }
  }
  GVMeta meta;
  std::memset(&meta, 0, sizeof(meta));
  meta.d = d;
  meta.ngroup = G;
  for (int i = 0; i < 3; ++i) meta.gdim[i] = i < d ? n[i] : 1;
  for (int g = 0; g < G; ++g) {
    meta.grp[g].off = gr[g].off;
    meta.grp[g].C = gr[g].C;
    for (int i = 0; i < 3; ++i) meta.grp[g].cs[i] = gr[g].cs[i];
    meta.grp[g].U = gr[g].U;
    for (int i = 0; i < d; ++i) meta.grp[g].W[i] = gr[g].isfree[i] ? nullptr : pg.P[gr[g].g][gr[g].c][i];
  }
  GVMeta* dmeta = (GVMeta*)tmp.alloc(sizeof(GVMeta));
  if (!dmeta) { h->err = "posterior: out of device memory"; return GPFVM_E_NOMEM; }
  if (hipMemcpyAsync(dmeta, &meta, sizeof(meta), hipMemcpyHostToDevice, s) != hipSuccess) {
    h->err = "posterior: copy failed";
    return GPFVM_E_HIP;
  }
  const dim3 grid(nblk(M)), block(256);
  switch (G) {
    case 1: hipLaunchKernelGGL(k_gv_direct<1>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 2: hipLaunchKernelGGL(k_gv_direct<2>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 3: hipLaunchKernelGGL(k_gv_direct<3>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 4: hipLaunchKernelGGL(k_gv_direct<4>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 5: hipLaunchKernelGGL(k_gv_direct<5>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 6: hipLaunchKernelGGL(k_gv_direct<6>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 7: hipLaunchKernelGGL(k_gv_direct<7>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 8: hipLaunchKernelGGL(k_gv_direct<8>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 9: hipLaunchKernelGGL(k_gv_direct<9>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 10: hipLaunchKernelGGL(k_gv_direct<10>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    case 11: hipLaunchKernelGGL(k_gv_direct<11>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
    default: hipLaunchKernelGGL(k_gv_direct<12>, grid, block, 0, s, (const GVMeta*)dmeta, M, nb, red); break;
  }
  if (hipGetLastError() != hipSuccess) { h->err = "posterior: launch failed"; return GPFVM_E_HIP; }
  return GPFVM_OK;
}

// W = G_bb^{-1} U for nrhs vectors (stored one after another) by library TRMMs: t = L^{-1} u,
// r = u - L t, t += L^{-1} r, then w = L^{-T} t, r = t - L^T w, w += L^{-T} r (the triangular
// solves with one residual correction each, as in the one-vector form).  U is overwritten.
static hipError_t ginv_trmm(const gpfvm_handle* h, int nrhs, double* U, double* T, double* W, double* R,
                            hipStream_t s) {
  const int nb = h->nb;
  const i64 len = (i64)nb * nrhs;
  hipError_t e;
  if ((e = trmm_vecs_lower(nb, nrhs, 0, h->Linv, U, T, s)) != hipSuccess) return e;     // t = Li u
  if ((e = trmm_vecs_lower(nb, nrhs, 0, h->L, T, R, s)) != hipSuccess) return e;        // r = L t
  if ((e = launch_axpby(len, 1.0, U, -1.0, R, s)) != hipSuccess) return e;             // r = u - r
  if ((e = trmm_vecs_lower(nb, nrhs, 0, h->Linv, R, W, s)) != hipSuccess) return e;     // (Li r)
  if ((e = launch_axpby(len, 1.0, W, 1.0, T, s)) != hipSuccess) return e;              // t += Li r
  if ((e = trmm_vecs_lower(nb, nrhs, 1, h->Linv, T, W, s)) != hipSuccess) return e;     // w = Li^T t
  if ((e = trmm_vecs_lower(nb, nrhs, 1, h->L, W, R, s)) != hipSuccess) return e;        // r = L^T w
  if ((e = launch_axpby(len, 1.0, T, -1.0, R, s)) != hipSuccess) return e;             // r = t - r
  if ((e = trmm_vecs_lower(nb, nrhs, 1, h->Linv, R, U, s)) != hipSuccess) return e;     // (Li^T r)
  return launch_axpby(len, 1.0, U, 1.0, W, s);                                          // w += Li^T r
}

extern "C" int gpfvm_posterior(gpfvm_handle* h, int dim, const int* n, const double* const* axis, double* mean,
                               double* var, void* stream) {
  if (!h) return GPFVM_E_INVALID;
  if (dim != h->d || !n || !axis || !mean) { h->err = "posterior: bad grid arguments"; return GPFVM_E_INVALID; }
  i64 M = 1;
  for (int i = 0; i < dim; ++i) {
    if (n[i] < 1 || !axis[i]) { h->err = "posterior: bad grid axis"; return GPFVM_E_INVALID; }
    for (int j = 0; j < n[i]; ++j)
      if (!std::isfinite(axis[i][j])) { h->err = "posterior: non-finite grid"; return GPFVM_E_INVALID; }
    M *= n[i];
  }
  if (!h->solved) { h->err = "posterior: no solve yet"; return GPFVM_E_STATE; }
  if (var && h->cg_only) {
    h->err = "posterior: a CG solve stores no directions; the variance needs method ITERGP";
    return GPFVM_E_STATE;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  const int d = h->d;
  const i64 N = h->N, Nc = h->Nc;
  const size_t T = h->pterms.size();
  Arena tmp;    // per-call allocations
  tmp.cache = h->arena.cache;
  auto fail = [&](int code, const std::string& m) { h->err = m; (void)hipStreamSynchronize(s); tmp.release(); return code; };
  // grid axes on the device
  double* gax[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < d; ++i) {
    gax[i] = (double*)tmp.alloc(n[i] * sizeof(double));
    if (!gax[i]) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
    if (hipMemcpyAsync(gax[i], axis[i], n[i] * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(GPFVM_E_HIP, "posterior: copy failed");
  }
  // grid-cell factors per term and dim, grid-point factors per point component and dim
  // (the component's per-point weights folded into its rows)
  std::vector<std::array<double*, 3>> Qg(T);
  for (size_t t = 0; t < T; ++t)
    for (int i = 0; i < d; ++i) {
      Qg[t][i] = (double*)tmp.alloc((size_t)n[i] * h->nc[i] * sizeof(double));
      if (!Qg[t][i]) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
      if (launch_factor(1, h->kq[i], 0, h->pterms[t].alpha[i], n[i], gax[i], h->nc[i], h->edges[i], h->ell[i], 1.0, Qg[t][i],
                        h->nc[i], s) != hipSuccess)
        return fail(GPFVM_E_HIP, "posterior: factor launch failed");
    }
  PGMeta pg;
  std::memset(&pg, 0, sizeof(pg));
  pg.d = d;
  pg.ngroup = (int)h->groups.size();
  for (int i = 0; i < d; ++i) pg.gdim[i] = n[i];
  for (size_t g = 0; g < h->groups.size(); ++g) {
    const Group& G = h->groups[g];
    pg.goff[g] = G.offset;
    pg.gcomp[g] = (int)G.comps.size();
    for (int i = 0; i < d; ++i) pg.gn[g][i] = G.n[i];
    double* ga[3] = {nullptr, nullptr, nullptr};
    for (int i = 0; i < d; ++i) {
      ga[i] = (double*)tmp.alloc(G.n[i] * sizeof(double));
      if (!ga[i]) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
      if (hipMemcpyAsync(ga[i], G.axis[i].data(), G.n[i] * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(GPFVM_E_HIP, "posterior: copy failed");
    }
    for (size_t c = 0; c < G.comps.size(); ++c)
      for (int i = 0; i < d; ++i) {
        const PointComp& C = G.comps[c];
        double* P = (double*)tmp.alloc((size_t)G.n[i] * n[i] * sizeof(double));
        if (!P) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
        // P[b][x] = d^beta_1 k(x_b, x), times the component's weight of point b
        if (launch_factor(2, h->kq[i], C.deriv[i], 0, G.n[i], ga[i], n[i], gax[i], h->ell[i], 1.0, P, n[i], s) !=
            hipSuccess)
          return fail(GPFVM_E_HIP, "posterior: factor launch failed");
        if (!C.w[i].empty()) {
          double* w = (double*)tmp.alloc(G.n[i] * sizeof(double));
          if (!w) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
          if (hipMemcpyAsync(w, C.w[i].data(), G.n[i] * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
              scale_rows_cols(P, G.n[i], n[i], w, nullptr, s) != hipSuccess)
            return fail(GPFVM_E_HIP, "posterior: weight scaling failed");
        }
        pg.P[g][c][i] = P;
      }
  }
  pg.goff[h->groups.size()] = h->nb;
  struct UserRange {
    const void* p;
    UserRange(const void* q, size_t n) : p(q) { register_range(q, n); }
    ~UserRange() { unregister_range(p); }
  } user_mean(mean, (size_t)M * h->nout * sizeof(double));
  double* alpha = (double*)tmp.alloc((size_t)h->n * sizeof(double));
  if (!alpha) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
  int rc = gpfvm_weights(h, alpha, s);
  if (rc) { tmp.release(); return rc; }
  // ---- variance buffers and the output-independent part of the direction term ----
  const int K = var ? h->iters : 0;
  const i64 widest = std::max<i64>(std::max<i64>(M, N), std::max(h->nb, 1));
  const int B = K > 0 ? (int)posterior_dir_batch(K, widest) : 0;
  double *red = nullptr, *P1 = nullptr, *P2 = nullptr, *Ub = nullptr, *Tb = nullptr, *Wb = nullptr, *Rb = nullptr,
         *Dbuf = nullptr;
  Plan pbp;
  if (var) {
    red = (double*)tmp.alloc((size_t)M * sizeof(double));
    if (!red) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
  }
  if (K > 0) {
    P1 = (double*)tmp.alloc((size_t)M * B * sizeof(double));
    P2 = h->nb > 0 ? (double*)tmp.alloc((size_t)M * B * sizeof(double)) : nullptr;
    Ub = h->nb > 0 ? (double*)tmp.alloc((size_t)h->nb * B * sizeof(double)) : nullptr;
    Tb = h->nb > 0 ? (double*)tmp.alloc((size_t)h->nb * B * sizeof(double)) : nullptr;
    Wb = h->nb > 0 ? (double*)tmp.alloc((size_t)h->nb * B * sizeof(double)) : nullptr;
    Rb = h->nb > 0 ? (double*)tmp.alloc((size_t)h->nb * B * sizeof(double)) : nullptr;
    Dbuf = (double*)tmp.alloc((size_t)N * B * sizeof(double));
    if (!P1 || !Dbuf || (h->nb > 0 && (!P2 || !Ub || !Tb || !Wb || !Rb)))
      return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
    if (h->nb > 0) {
      rc = compile_kron_list(h->op_bp, F64, B, Dbuf, N, Ub, h->nb, h->cellc, h->cellc, 0.0, nullptr, 0, 0, tmp, s, pbp,
                             h->err);
      if (rc) { tmp.release(); return rc; }
    }
  }
  // with all directions in one batch, G_bb^{-1} G_bp D is shared by every output
  bool wb_ready = false;
  std::vector<std::unique_ptr<PGMeta>> pg_keep;
  for (int o = 0; o < h->nout; ++o) {
    double* mean_o = mean + (i64)o * M;
    double* var_o = var ? var + (i64)o * M : nullptr;
    // operators for output o: K_*p (volumes -> grid), K_*b (points -> grid)
    KronOp gp;
    gp.d = d;
    for (int i = 0; i < d; ++i) { gp.in_shape[i] = h->nc[i]; gp.out_shape[i] = n[i]; }
    gp.in_len = N;
    for (size_t t = 0; t < T; ++t) {
      if (h->pterms[t].out != o) continue;
      KronTerm k{};
      for (int i = 0; i < d; ++i) { k.M[i] = Qg[t][i]; k.ld[i] = h->nc[i]; }
      k.alpha = h->sfo[o] * h->pterms[t].coef;
      k.rscale = h->pterms[t].cellwise;
      k.in_off = (i64)h->pterms[t].eq * Nc;
      gp.terms.push_back(k);
    }
    std::vector<KronOp> gb;
    for (size_t g = 0; g < h->groups.size(); ++g) {
      const Group& G = h->groups[g];
      KronOp op;
      op.d = d;
      for (int i = 0; i < d; ++i) { op.in_shape[i] = G.n[i]; op.out_shape[i] = n[i]; }
      op.in_len = h->nb;
      for (size_t c = 0; c < G.comps.size(); ++c) {
        pg.pc[g][c] = G.comps[c].out == o ? h->sfo[o] * G.comps[c].coef : 0.0;
        if (G.comps[c].out != o) continue;
        KronTerm k{};
        for (int i = 0; i < d; ++i) { k.M[i] = pg.P[g][c][i]; k.ld[i] = n[i]; k.trans[i] = 1; }
        k.alpha = h->sfo[o] * G.comps[c].coef;
        k.in_off = G.offset;
        op.terms.push_back(k);
      }
      if (!op.terms.empty()) gb.push_back(op);
    }
    // ---- mean = K_*b alpha_b + K_*p alpha_p ----
    if (gp.terms.empty()) {
      if (launch_fill(mean_o, 0.0, M, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: fill failed");
    } else {
      Plan pm;
      std::vector<KronOp> ops{gp};
      rc = compile_kron_list(ops, F64, 1, alpha + h->nb, N, mean_o, M, h->cellc, h->cellc, 0.0, nullptr, 0, 1, tmp, s,
                             pm, h->err);
      if (rc) { tmp.release(); return rc; }
      if (run_plan(pm, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: mean plan failed");
    }
    if (!gb.empty()) {
      Plan pmb;
      rc = compile_kron_list(gb, F64, 1, alpha, h->nb, mean_o, M, nullptr, nullptr, 1.0, nullptr, 0, 1, tmp, s, pmb,
                             h->err);
      if (rc) { tmp.release(); return rc; }
      if (run_plan(pmb, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: mean plan failed");
    }
    if (!var) continue;
    // ---- variance = s_o - ||L^{-1} k_b(x)||^2 - sum_j (w_j(x))^2 / eta_j ----
    if (launch_fill(red, 0.0, M, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: fill failed");
    if (h->nb > 0 && !gb.empty()) {
      // this output's coefficients, from a host copy that outlives the queued upload
      pg_keep.push_back(std::make_unique<PGMeta>(pg));
      PGMeta* dpg = (PGMeta*)tmp.alloc(sizeof(PGMeta));
      if (!dpg) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
      if (hipMemcpyAsync(dpg, pg_keep.back().get(), sizeof(pg), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(GPFVM_E_HIP, "posterior: copy failed");
      const int grc = grouped_point_var(h, pg, n, M, red, tmp, s);
      if (grc != 1 && grc != GPFVM_OK) return fail(grc, h->err);
      if (grc == 1) {
        const i64 chunk = posterior_chunk(h->nb, M);
        double* KB = (double*)tmp.alloc((size_t)h->nb * chunk * sizeof(double));
        double* TT = (double*)tmp.alloc((size_t)h->nb * chunk * sizeof(double));
        double* CP = (double*)tmp.alloc((size_t)COLSQ_MAX_CHUNKS * chunk * sizeof(double));
        if (!KB || !TT || !CP) return fail(GPFVM_E_NOMEM, "posterior: out of device memory");
        for (i64 x0 = 0; x0 < M; x0 += chunk) {
          const i64 nx = std::min(chunk, M - x0);
          hipLaunchKernelGGL(k_point_grid, dim3(nblk((i64)h->nb * nx)), dim3(256), 0, s, (const PGMeta*)dpg, h->nb, x0,
                             nx, KB);
          // T = L^{-1} KB by the explicit inverse (a library TRMM).  Its forward error, about
          // cond(L) eps relative, is that of a triangular solve, so ||T||^2 needs no residual
          // correction here (the solver's operator does: there the products must stay
          // consistent over hundreds of iterations).
          if (trmm_rows_left_lower(h->nb, (int)nx, 1.0, h->Linv, h->nb, KB, (int)nx, TT, (int)nx, s) != hipSuccess)
            return fail(GPFVM_E_HIP, "posterior: triangular product failed");
          const int R = colsq_chunks(h->nb, nx);
          hipLaunchKernelGGL(k_colsq_part, dim3((unsigned)((nx + 63) / 64), (unsigned)R), dim3(256), 0, s, (i64)h->nb,
                             nx, (const double*)TT, CP);
          hipLaunchKernelGGL(k_colsq_finish, dim3(nblk(nx)), dim3(256), 0, s, nx, R, (const double*)CP, red + x0);
        }
      }
    }
    if (K > 0) {
      Plan pgp, pgb;
      const bool have_gp = !gp.terms.empty(), have_gb = h->nb > 0 && !gb.empty();
      if (have_gp) {
        std::vector<KronOp> ops{gp};
        rc = compile_kron_list(ops, F64, B, Dbuf, N, P1, M, h->cellc, h->cellc, 0.0, nullptr, 0, 1, tmp, s, pgp, h->err);
        if (rc) { tmp.release(); return rc; }
      }
      if (have_gb) {
        rc = compile_kron_list(gb, F64, B, Wb, h->nb, P2, M, nullptr, nullptr, 0.0, nullptr, 0, 1, tmp, s, pgb, h->err);
        if (rc) { tmp.release(); return rc; }
      }
      if (!have_gp && launch_fill(P1, 0.0, M * B, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: fill failed");
      const bool one_batch = K <= B;
      for (int j0 = 0; j0 < K; j0 += B) {
        const int nr = std::min(B, K - j0);
        if (!(one_batch && wb_ready)) {
          if (hipMemcpyAsync(Dbuf, h->Dd + (i64)j0 * N, (size_t)nr * N * sizeof(double), hipMemcpyDeviceToDevice,
                             s) != hipSuccess)
            return fail(GPFVM_E_HIP, "posterior: copy failed");
          if (nr < B && launch_fill(Dbuf + (i64)nr * N, 0.0, (i64)(B - nr) * N, s) != hipSuccess)
            return fail(GPFVM_E_HIP, "posterior: fill failed");
        }
        if (have_gp && run_plan(pgp, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: plan failed");
        if (have_gb) {
          if (!(one_batch && wb_ready)) {
            if (run_plan(pbp, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: plan failed");
            if (ginv_trmm(h, B, Ub, Tb, Wb, Rb, s) != hipSuccess)
              return fail(GPFVM_E_HIP, "posterior: triangular products failed");
            wb_ready = one_batch;
          }
          if (run_plan(pgb, s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: plan failed");
        }
        hipLaunchKernelGGL(k_sub_sq_acc, dim3(nblk(M)), dim3(256), 0, s, M, nr, (const double*)P1,
                           (const double*)(have_gb ? P2 : nullptr), (const double*)(h->eta + j0), red);
      }
    }
    hipLaunchKernelGGL(k_var_final, dim3(nblk(M)), dim3(256), 0, s, M, h->sfo[o], (const double*)red, var_o);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(GPFVM_E_HIP, "posterior: kernel failed");
  tmp.release();
  return GPFVM_OK;
}


// ---------------------------------------------------------------------------
// Batched solve of R problems that share the handle's operator: the same
// grid, kernel, PDE and point layout, different point data (serving requests
// of one grid size).  Each problem runs its own IterGP recurrence (its own
// directions, eta and weights, float64, two projection passes, residual
// replacement every `replace_every`), in lockstep: one batched iteration
// applies the shared volume-system operator to all R actions at once (the
// nrhs = R plan: grouped GEMM launches, the point block as GEMM-form
// triangular products), and every projection, update and dot product of all
// problems runs as one launch with a batch dimension.  A problem that has
// converged keeps its state; its share of the later launches does nothing.
// ---------------------------------------------------------------------------
int gpfvm::batch_solve(gpfvm_handle* h, int R, const double* yobs_host, double tol, int max_iter, int check_every,
                       int replace_every, hipStream_t s, std::vector<BatchResult>& out) {
  if (R < 1 || max_iter < 1 || max_iter > h->max_iter) { h->err = "batch: bad size"; return GPFVM_E_INVALID; }
  if (h->multi) { h->err = "batch: batched solves take single-output problems"; return GPFVM_E_INVALID; }
  h->stream = s;
  const i64 N = h->N, n = h->n, nb = h->nb, cap = h->max_iter;
  gpfvm_sop* so = nullptr;
  int rc = get_sop(h, R, F64, &so);
  if (rc) return rc;
  GpfvmBatch& B = h->batch;
  B = GpfvmBatch();
  B.R = R;
  const int n_eta = (int)((N + 63) / 64), n_rr = (int)nblk(N);
  const i64 ucap = 2 * cap + ROWS_DOT_TARGET, pstride = n_eta + 2 * (i64)n_rr;
  auto A = [&](size_t bytes) { return h->arena.alloc(bytes); };
  B.yobs = (double*)A((size_t)R * n * 8);
  B.bS = (double*)A((size_t)R * N * 8);
  B.v = (double*)A((size_t)R * N * 8);
  B.Dd = (double*)A((size_t)R * cap * N * 8);
  B.Qd = (double*)A((size_t)R * cap * N * 8);
  B.eta = (double*)A((size_t)R * cap * 8);
  double* r = (double*)A((size_t)R * N * 8);
  double* d = (double*)A((size_t)R * N * 8);
  double* w = (double*)A((size_t)R * N * 8);
  double* coef = (double*)A((size_t)R * ucap * 8);
  double* dotp = (double*)A((size_t)R * DOT_PARTIALS * 8);
  double* scal = (double*)A((size_t)R * 64 * 8);
  int* flag = (int*)A((size_t)R * 16 * sizeof(int));
  double* part = (double*)A((size_t)R * pstride * 8);
  if (!B.yobs || !B.bS || !B.v || !B.Dd || !B.Qd || !B.eta || !r || !d || !w || !coef || !dotp || !scal || !flag ||
      !part) {
    h->err = "out of device memory (batched solve)";
    return GPFVM_E_NOMEM;
  }
  double* X = (double*)so->X;
  const double* Y = (const double*)so->Y;
  BatchStrides bs;
  bs.M = cap * N; bs.v = N; bs.u = ucap; bs.eta = cap; bs.part = pstride; bs.scal = 64; bs.flag = 16;
  BatchStrides bsd;                               // dots: vectors and scalars only
  bsd.v = N; bsd.scal = 64;
  // data, and b_r = y_p - G_pb G_bb^{-1} y_b,r for all problems with the nrhs = R plans
  HIPCHK(h, hipMemcpyAsync(B.yobs, yobs_host, (size_t)R * n * 8, hipMemcpyHostToDevice, s));
  HIPCHK(h, launch_fill(B.v, 0.0, (i64)R * N, s));
  HIPCHK(h, launch_fill(B.eta, 1.0, (i64)R * cap, s));
  for (int z = 0; z < R; ++z)
    HIPCHK(h, hipMemcpyAsync(B.bS + (i64)z * N, B.yobs + (i64)z * n + nb, N * 8, hipMemcpyDeviceToDevice, s));
  if (nb > 0) {
    for (int z = 0; z < R; ++z)
      HIPCHK(h, hipMemcpyAsync((double*)so->U + (i64)z * nb, B.yobs + (i64)z * n, nb * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, run_stages(so->ginv, s));
    HIPCHK(h, launch_fill((double*)so->Y, 0.0, (i64)R * N, s));
    HIPCHK(h, run_plan(so->pb, s));
    HIPCHK(h, launch_axpby((i64)R * N, 1.0, Y, 1.0, B.bS, s));
  }
  // r = b - S v (v = 0), X = r; b.b; the stopping test of every problem
  HIPCHK(h, hipMemsetAsync(flag, 0, (size_t)R * 16 * sizeof(int), s));
  HIPCHK(h, hipMemcpyAsync(X, B.v, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, apply_sop(h, so, s));
  HIPCHK(h, launch_dot(N, B.bS, B.bS, dotp, scal + 3, s, R, bsd));
  {
    std::vector<double> t2(R * 64, 0.0);
    HIPCHK(h, hipMemcpyAsync(t2.data(), scal, (size_t)R * 64 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    for (int z = 0; z < R; ++z) t2[z * 64 + 4] = tol * tol;
    HIPCHK(h, hipMemcpyAsync(scal, t2.data(), (size_t)R * 64 * 8, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  hipLaunchKernelGGL(k_resid2, dim3(nblk(N), R), dim3(256), 0, s, N, (const double*)B.bS, Y, r, X,
                     (const int*)flag, N, (i64)16);
  HIPCHK(h, launch_dot_check(N, r, dotp, scal, flag, max_iter, s, R, bs));
  double* eta_p = part;
  double* rr_a = part + n_eta;
  double* rr_b = rr_a + n_rr;
  double* rr_prev = nullptr;
  std::vector<int> hflag((size_t)R * 16, 0);
  int i = 0;
  while (i < max_iter) {
    const int end = std::min(max_iter, i + std::max(1, check_every));
    for (; i < end; ++i) {
      HIPCHK(h, apply_sop(h, so, s));                                 // Y = S X, all problems
      if (i > 0) {
        const int nch = rows_dot_chunks(i, N);
        HIPCHK(h, launch_rows_dot(i, N, B.Dd, Y, coef, s, nullptr, R, bs));
        HIPCHK(h, launch_cols_update(i, N, B.Dd, coef, nch, B.eta, X, d, nullptr, B.Qd, Y, w, s, nullptr, nullptr,
                                     R, bs));
        HIPCHK(h, launch_rows_dot(i, N, B.Dd, w, coef, s, nullptr, R, bs));
        HIPCHK(h, launch_cols_update(i, N, B.Dd, coef, nch, B.eta, d, d, nullptr, B.Qd, w, w, s, eta_p, nullptr,
                                     R, bs));
      } else {
        HIPCHK(h, hipMemcpyAsync(d, X, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(h, hipMemcpyAsync(w, Y, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(h, launch_dot(N, w, d, dotp, scal + 1, s, R, bsd));    // eta = d^T S d
      }
      const bool replace = (i + 1) % std::max(1, replace_every) == 0;
      double* rr_next = replace ? nullptr : (rr_prev == rr_a ? rr_b : rr_a);
      const bool upd_inl = update_inline(N);
      if (!upd_inl && (i > 0 || rr_prev))
        hipLaunchKernelGGL(k_update_sums, dim3(1, R), dim3(256), 0, s, (const double*)rr_prev, n_rr,
                           (const double*)(i > 0 ? eta_p : nullptr), n_eta, scal, bs);
      hipLaunchKernelGGL(k_update2x, dim3(nblk(N), R), dim3(256), 0, s, N, (const double*)d, (const double*)w, B.v,
                         r, X, B.Dd + (i64)i * N, B.Qd + (i64)i * N, B.eta + i, scal, flag,
                         (const double*)(i > 0 ? eta_p : nullptr), n_eta, (const double*)rr_prev, n_rr, rr_next, bs,
                         nullptr, 0, upd_inl ? 1 : 0);
      rr_prev = rr_next;
      if (replace) {
        HIPCHK(h, hipMemcpyAsync(X, B.v, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(h, apply_sop(h, so, s));
        hipLaunchKernelGGL(k_resid2, dim3(nblk(N), R), dim3(256), 0, s, N, (const double*)B.bS, Y, r, X,
                           (const int*)flag, N, (i64)16);
        HIPCHK(h, hipMemcpyAsync(X, r, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(h, launch_dot_check(N, r, dotp, scal, flag, max_iter, s, R, bs));
      }
    }
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(hflag.data(), flag, (size_t)R * 16 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    bool all = true;
    for (int z = 0; z < R; ++z) all = all && hflag[(size_t)z * 16] != 0;
    if (all) break;
  }
  // explicit residual of every problem
  HIPCHK(h, hipMemcpyAsync(X, B.v, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, apply_sop(h, so, s));
  HIPCHK(h, hipMemcpyAsync(r, B.bS, (size_t)R * N * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, launch_axpby((i64)R * N, -1.0, Y, 1.0, r, s));
  HIPCHK(h, launch_dot(N, r, r, dotp, scal + 8, s, R, bsd));
  std::vector<double> hs((size_t)R * 64);
  HIPCHK(h, hipMemcpyAsync(hs.data(), scal, (size_t)R * 64 * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  out.assign(R, BatchResult());
  B.iters.assign(R, 0);
  for (int z = 0; z < R; ++z) {
    B.iters[z] = hflag[(size_t)z * 16 + 1];
    out[z].iters = B.iters[z];
    out[z].state = hflag[(size_t)z * 16];
    const double bb = hs[(size_t)z * 64 + 3], rr = hs[(size_t)z * 64 + 8];
    out[z].rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  }
  return GPFVM_OK;
}

// Posterior of problem z of the last batched solve: the handle's solver state
// is pointed at that problem's slices for the call.
int gpfvm::batch_posterior(gpfvm_handle* h, int z, int dim, const int* n, const double* const* axis, double* mean,
                           double* var, hipStream_t s) {
  GpfvmBatch& B = h->batch;
  if (z < 0 || z >= B.R) { h->err = "batch: no such problem"; return GPFVM_E_INVALID; }
  const i64 N = h->N, cap = h->max_iter;
  double *v0 = h->v, *D0 = h->Dd, *Q0 = h->Qd, *e0 = h->eta, *y0 = h->yobs, *b0 = h->bS;
  const int it0 = h->iters;
  const bool s0 = h->solved, x0 = h->sd_exact, c0 = h->cg_only;
  h->v = B.v + (i64)z * N;
  h->Dd = B.Dd + (i64)z * cap * N;
  h->Qd = B.Qd + (i64)z * cap * N;
  h->eta = B.eta + (i64)z * cap;
  h->yobs = B.yobs + (i64)z * h->n;
  h->bS = B.bS + (i64)z * N;
  h->iters = B.iters[z];
  h->solved = true;
  h->sd_exact = true;
  h->cg_only = false;
  const int rc = gpfvm_posterior(h, dim, n, axis, mean, var, s);
  h->v = v0; h->Dd = D0; h->Qd = Q0; h->eta = e0; h->yobs = y0; h->bS = b0; h->iters = it0;
  h->solved = s0; h->sd_exact = x0; h->cg_only = c0;
  return rc;
}
