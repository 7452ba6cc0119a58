// Dense pieces of the hot path: Gram tiles generated entry-by-entry from the
// 1-D factor tiles (Sec. 4.1 eq. kronecker-structure; Sec. 2.2 IBVP block
// layout), the float64 blocked Cholesky of the point block and its triangular
// inverse (Sec. 4.2, Cholesky preconditioner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>

#include "common.h"
#include "internal.h"

namespace gpfvm {

// ---------------------------------------------------------------------------
// Dense Gram block: entry (r, c) of G = L k L' + Sigma in observation order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void unflatten(i64 idx, int d, const int* shape, int* out) {
  for (int i = d - 1; i >= 0; --i) {
    out[i] = (int)(idx % shape[i]);
    idx /= shape[i];
  }
}

__device__ __forceinline__ int find_group(const GramMeta& G, i64 r) {
  int g = 0;
  while (g + 1 < G.ngroup && G.goff[g + 1] <= r) ++g;
  return g;
}

__global__ void k_gram_block(const GramMeta* __restrict__ meta, i64 r0, i64 nr, i64 c0, i64 nc,
                             double* __restrict__ out, i64 ld) {
  const GramMeta& G = *meta;
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nr * nc) return;
  const i64 r = r0 + idx / nc, c = c0 + idx % nc;
  const int d = G.d;
  double v = 0;
  int ir[3] = {0, 0, 0}, ic[3] = {0, 0, 0};
  const bool rp = r < G.nb, cp = c < G.nb;
  if (rp && cp) {                      // point - point: component pairs on the same output
    const int g1 = find_group(G, r), g2 = find_group(G, c);
    unflatten(r - G.goff[g1], d, G.gn[g1], ir);
    unflatten(c - G.goff[g2], d, G.gn[g2], ic);
    for (int c1 = 0; c1 < G.gcomp[g1]; ++c1)
      for (int c2 = 0; c2 < G.gcomp[g2]; ++c2) {
        const double a = G.pcoef[g1][c1][g2][c2];
        if (a == 0.0) continue;
        double p = a;
        for (int i = 0; i < d; ++i) p *= G.Pp[g1][c1][g2][c2][i][(i64)ir[i] * G.gn[g2][i] + ic[i]];
        v += p;
      }
    if (r == c) v += G.gnoise[g1];
  } else if (rp != cp) {               // point - volume (symmetric): the volume's equation
    const i64 pr = rp ? r : c, vo = (rp ? c : r) - G.nb;
    const int g = find_group(G, pr);
    const int e = (int)(vo / G.Nc);
    const i64 vc = vo - (i64)e * G.Nc;
    unflatten(pr - G.goff[g], d, G.gn[g], ir);
    unflatten(vc, d, G.nc, ic);
    for (int k = 0; k < G.gcomp[g]; ++k)
      for (int t = 0; t < G.nterm; ++t) {
        if (G.teq[t] != e || G.qcoef[g][k][t] == 0.0) continue;
        double p = G.qcoef[g][k][t];
        if (G.tcw[t]) p *= G.cellc[vc];
        for (int i = 0; i < d; ++i) p *= G.Qp[g][k][t][i][(i64)ir[i] * G.nc[i] + ic[i]];
        v += p;
      }
  } else {                             // volume - volume: merged terms of the two equations
    const i64 vr0 = r - G.nb, vc0 = c - G.nb;
    const int er = (int)(vr0 / G.Nc), ec = (int)(vc0 / G.Nc);
    const i64 vr = vr0 - (i64)er * G.Nc, vc = vc0 - (i64)ec * G.Nc;
    unflatten(vr, d, G.nc, ir);
    unflatten(vc, d, G.nc, ic);
    for (int t = 0; t < G.ngterm; ++t) {
      if (G.ge1[t] != er || G.ge2[t] != ec) continue;
      double p = G.gcoef[t];
      if (G.gl[t]) p *= G.cellc[vr];
      if (G.gr[t]) p *= G.cellc[vc];
      for (int i = 0; i < d; ++i) p *= G.Dp[i][G.gm[t][i]][(i64)ir[i] * G.nc[i] + ic[i]];
      v += p;
    }
    if (r == c) v += G.sig_pde;
  }
  out[(idx / nc) * ld + (idx % nc)] = v;
}

hipError_t launch_gram_block(const GramMeta* meta, i64 r0, i64 nr, i64 c0, i64 nc, double* out, i64 ld,
                             hipStream_t s) {
  const i64 tot = nr * nc;
  if (tot == 0) return hipSuccess;
  k_gram_block<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(meta, r0, nr, c0, nc, out, ld);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagonal block of the blocked Cholesky: factor the nb x nb block at (k0,k0)
// in LDS, write L_kk back and the inverse of L_kk into dinv (NB x NB, row-major).
// Sets *flag = 1 + k0 if a pivot of the block is not positive.
// ---------------------------------------------------------------------------
constexpr int NB = 64;

__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ A, i64 ld, int k0, int nb,
                                                    double* __restrict__ dinv, int* __restrict__ flag) {
  __shared__ double L[NB][NB + 1];
  __shared__ double V[NB][NB + 1];
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;     // 16 x 16 threads, 4 x 4 elements each
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    L[i][j] = (i < nb && j < nb) ? A[(i64)(k0 + i) * ld + k0 + j] : (i == j ? 1.0 : 0.0);
    V[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (*flag != 0) return;            // an earlier block already failed
  // right-looking Cholesky: column j is scaled, then the trailing lower triangle
  // takes the rank-1 update, each thread on its fixed 4 x 4 set of elements
  int bad = 0;
  for (int j = 0; j < nb; ++j) {
    const double p = L[j][j];          // the same value in every thread
    if (!(p > 0.0)) { bad = 1; break; }
    const double dj = sqrt(p);
    __syncthreads();                   // every thread has read the pivot
    for (int i = j + t; i < nb; i += blockDim.x) L[i][j] = (i == j) ? dj : L[i][j] / dj;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = ty + 16 * a, c = tx + 16 * b;
        if (i < nb && c > j && c <= i) L[i][c] -= L[i][j] * L[c][j];
      }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) atomicCAS(flag, 0, 1 + k0);
    return;
  }
  // inverse by forward elimination on [L | I]: row j of V is divided by L[j][j],
  // then subtracted from the rows below with multipliers L[i][j]
  for (int j = 0; j < nb; ++j) {
    const double dj = L[j][j];
    if (t <= j) V[j][t] /= dj;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = ty + 16 * a, c = tx + 16 * b;
        if (i > j && i < nb && c <= j) V[i][c] -= L[i][j] * V[j][c];
      }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    if (i < nb && j < nb) A[(i64)(k0 + i) * ld + k0 + j] = (j <= i) ? L[i][j] : 0.0;
    dinv[e] = (i < nb && j < nb && j <= i) ? V[i][j] : 0.0;
  }
}

// dst[i][j] += alpha src[i][j] over an r x c block (row-major, leading dimensions sld, dld),
// for blockIdx.y blocks src_bs and dst_bs elements apart
__global__ void k_axpy2d(const double* __restrict__ src, i64 sld, double* __restrict__ dst, i64 dld, i64 r, i64 c,
                         double alpha, i64 src_bs = 0, i64 dst_bs = 0) {
  const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * c) return;
  src += blockIdx.y * src_bs;
  dst += blockIdx.y * dst_bs;
  const i64 i = t / c, j = t % c;
  dst[i * dld + j] += alpha * src[i * sld + j];
}

__global__ void k_copy2d(const double* __restrict__ src, i64 sld, double* __restrict__ dst, i64 dld,
                         i64 rows, i64 cols) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const i64 r = idx / cols, c = idx % cols;
  dst[r * dld + c] = src[r * sld + c];
}

__global__ void k_zero_upper(double* A, i64 ld, i64 n) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const i64 r = idx / n, c = idx % n;
  if (c > r) A[r * ld + c] = 0.0;
}

static void gemm_desc_init(GemmDesc& D) { std::memset(&D, 0, sizeof(D)); }

// Append a plain descriptor C = alpha * A * B + beta * C (single batch).
static GemmDesc mk_desc(double* C, i64 ldc, const double* A, i64 a_rs, i64 a_cs, const double* B, i64 b_rs,
                        i64 b_cs, int M, int N, int K, double alpha, double beta, int lower_only,
                        int tri) {
  GemmDesc D;
  gemm_desc_init(D);
  D.C = C; D.c_rs = ldc; D.c_cs = 1;
  D.M = M; D.N = N; D.batch = 1; D.nseg = 1;
  D.beta = beta; D.lower_only = lower_only;
  Seg& S = D.seg[0];
  S.A = A; S.a_rs = a_rs; S.a_cs = a_cs;
  S.B = B; S.b_rs = b_rs; S.b_cs = b_cs;
  S.K = K; S.alpha = alpha; S.tri = tri;
  return D;
}

// Extent in bytes of an operand addressed as base + r*rs + c*cs + b*bs.
static bool extent_ok(const void* base, i64 rows, i64 cols, i64 batch, i64 rs, i64 cs, i64 bs, size_t es) {
  if (!base) return false;
  if (rows <= 0 || cols <= 0 || batch <= 0) return true;
  if (rs < 0 || cs < 0 || bs < 0) return false;
  const i64 last = (rows - 1) * rs + (cols - 1) * cs + (batch - 1) * bs;
  return range_ok(base, (size_t)(last + 1) * es);
}

// Host-side bounds check of every operand of a descriptor.
bool desc_in_bounds(const GemmDesc& D, size_t es) {
  if (D.nseg < 1 || D.nseg > MAXSEG || D.M < 0 || D.N < 0 || D.batch < 1) return false;
  if (!extent_ok(D.C, D.M, D.N, D.batch, D.c_rs, D.c_cs, D.c_bs, es)) return false;
  if (D.escale && !extent_ok(D.escale, D.M, D.N, D.batch, D.e_rs, D.e_cs, D.e_bs, sizeof(double))) return false;
  if (D.X && !extent_ok(D.X, D.M, D.N, D.batch, D.x_rs, D.x_cs, D.x_bs, es)) return false;
  for (int g = 0; g < D.nseg; ++g) {
    const Seg& S = D.seg[g];
    if (S.K < 0 || S.slot < 0 || S.slot > 1 || S.tri < 0 || S.tri > 4) return false;
    if (!extent_ok(S.A, D.M, S.K, D.batch, S.a_rs, S.a_cs, S.a_bs, es)) return false;
    if (!extent_ok(S.B, S.K, D.N, D.batch, S.b_rs, S.b_cs, S.b_bs, es)) return false;
  }
  return true;
}

// Pick the kernel of a stage (sizes measured on the advection-diffusion and
// wave volume operators).  Stages with at least 256 output tiles of 64x64 run
// on the 64x64 LDS-tiled kernel whatever their K.  Below that, long
// reductions (K beyond 2048: GEMV-shaped projections, point-block products
// with few right-hand sides) go to the split-K kernel, whose four wavefronts
// share the K range of a 32x32 tile, and short ones to the LDS-tiled kernel
// with its K range split over wavefront groups: 32x32 tiles and four groups,
// or, when that leaves fewer than 128 workgroups (one-right-hand-side mode
// products), 16x16 tiles and eight groups, for four times the workgroups and
// half the chunks in each one's sequential K loop.
void choose_kernel(Stage& st) {
  st.kind = GEMM_SPLITK;
  st.slot1 = 0;
  if (st.descs.empty()) return;
  i64 tiles64 = 0, tiles32 = 0, kmax = 0;
  for (auto& D : st.descs) {
    i64 ksum = 0;
    for (int g = 0; g < D.nseg; ++g) {
      ksum += D.seg[g].K;
      if (D.seg[g].slot) st.slot1 = 1;
    }
    kmax = std::max(kmax, ksum);
    tiles64 += (i64)((D.M + 63) / 64) * ((D.N + 63) / 64) * D.batch;
    tiles32 += (i64)((D.M + 31) / 32) * ((D.N + 31) / 32) * D.batch;
  }
  if (tiles64 >= 256) st.kind = GEMM_LDS64;
  else if (kmax <= 2048) st.kind = tiles32 < 128 ? GEMM_LDS16 : GEMM_LDS32;
}

// Upload a list of stages whose descriptors are consecutive in one buffer.
hipError_t upload_stages(std::vector<Stage>& stages, Arena& arena, hipStream_t s, Elt elt) {
  const size_t es = (elt == F64) ? sizeof(double) : sizeof(float);
  for (auto& st : stages)
    for (auto& D : st.descs)
      if (!desc_in_bounds(D, es)) return hipErrorInvalidValue;
  size_t total = 0;
  for (auto& st : stages) total += st.descs.size();
  if (total == 0) return hipSuccess;
  GemmDesc* dev = (GemmDesc*)arena.alloc(total * sizeof(GemmDesc));
  if (!dev) return hipErrorOutOfMemory;
  std::vector<GemmDesc> host;
  host.reserve(total);
  for (auto& st : stages) {
    // a mode product that contracts to a single output row or column uses 1/64 of a 64x64
    // MFMA tile: such descriptors go to the end and run on the thin kernel
    st.nthin = 0;
    st.thin_outputs = 0;
    if (elt != F32B) {
      auto thin = [](const GemmDesc& D) {
        return (D.M == 1 || D.N == 1) && D.nseg == 1 && !D.escale && !D.X && D.beta == 0.0 && D.seg[0].tri == 0 &&
               D.seg[0].slot == 0 && D.seg[0].K <= 4096;
      };
      std::stable_partition(st.descs.begin(), st.descs.end(), [&](const GemmDesc& D) { return !thin(D); });
      for (auto& D : st.descs)
        if (thin(D)) ++st.nthin;
    }
    std::vector<GemmDesc> thin_descs(st.descs.end() - st.nthin, st.descs.end());
    st.descs.resize(st.descs.size() - st.nthin);
    choose_kernel(st);
    if (elt == F32B) {               // split-bfloat16 GEMM: 64x64 tiles where there are enough, else 32x32
      i64 t64 = 0;
      for (auto& D : st.descs) t64 += (i64)((D.M + 63) / 64) * ((D.N + 63) / 64) * D.batch;
      st.kind = t64 >= 256 ? GEMM_BF16S64 : GEMM_BF16S32;
    }
    st.tiles = 0;
    for (auto& D : st.descs) {
      const int t = (st.kind == GEMM_LDS64 || st.kind == GEMM_BF16S64) ? 64 : st.kind == GEMM_LDS16 ? 16 : 32;
      D.tiles_m = (D.M + t - 1) / t;
      D.tiles_n = (D.N + t - 1) / t;
      D.tile_begin = st.tiles;
      st.tiles += (i64)D.tiles_m * D.tiles_n * D.batch;
    }
    for (auto& D : thin_descs) {
      D.tile_begin = st.thin_outputs;
      st.thin_outputs += (i64)D.M * D.N * D.batch;
      st.descs.push_back(D);
    }
    st.d_descs = dev + host.size();
    host.insert(host.end(), st.descs.begin(), st.descs.end());
  }
  hipError_t e = hipMemcpyAsync(dev, host.data(), total * sizeof(GemmDesc), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Blocked right-looking Cholesky of the n x n matrix A (row-major, lower),
// then L^{-1} into Linv.  Returns GPFVM_OK / GPFVM_E_NOTPD / GPFVM_E_HIP.
//
// The columns go in panels of PANEL = 8 blocks of 64.  Inside a panel each
// 64-column block is factored (diagonal block in LDS, explicit inverse of it),
// its rows below are solved with that inverse, and only the rest of the panel
// takes the block's rank-64 update; the trailing matrix takes the panel's
// rank-512 update at once (a library SYRK).  Same arithmetic as updating the
// whole trailing matrix after every block, with one eighth of its traffic.
constexpr int PANEL = 8 * NB;
int cholesky_and_inverse(double* A, double* Linv, int n, Arena& arena, hipStream_t s, std::string& err) {
  if (n == 0) return GPFVM_OK;
  const int nblk = (n + NB - 1) / NB;
  double* dinv = (double*)arena.alloc((size_t)nblk * NB * NB * sizeof(double));
  double* panel = (double*)arena.alloc((size_t)n * NB * sizeof(double));
  int* flag = (int*)arena.alloc(sizeof(int));
  if (!dinv || !panel || !flag) { err = "out of device memory (Cholesky workspace)"; return GPFVM_E_NOMEM; }
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return GPFVM_E_HIP;

  // descriptors: per block k, the solve of the rows below it and the update of the rest of its panel
  std::vector<Stage> st(2 * nblk);
  for (int k = 0; k < nblk; ++k) {
    const int k0 = k * NB, nbk = std::min(NB, n - k0), r0 = k0 + nbk, mr = n - r0;
    const int pe = std::min(n, (k0 / PANEL + 1) * PANEL), pc = pe - r0;
    if (mr > 0)       // L_rows = panel_copy * Dinv_k^T
      st[2 * k].descs.push_back(mk_desc(A + (i64)r0 * n + k0, n, panel, NB, 1, dinv + (i64)k * NB * NB, 1, NB,
                                        mr, nbk, nbk, 1.0, 0.0, 0, 0));
    if (pc > 0)       // A[r0:, r0:pe] -= L_rows L_rows[0:pc]^T (lower tiles)
      st[2 * k + 1].descs.push_back(mk_desc(A + (i64)r0 * n + r0, n, A + (i64)r0 * n + k0, n, 1,
                                            A + (i64)r0 * n + k0, 1, n, mr, pc, nbk, -1.0, 1.0, 1, 0));
  }
  if (upload_stages(st, arena, s) != hipSuccess) { err = "descriptor upload failed"; return GPFVM_E_HIP; }
  for (int k = 0; k < nblk; ++k) {
    const int k0 = k * NB, nbk = std::min(NB, n - k0), r0 = k0 + nbk, mr = n - r0;
    const int p0 = (k0 / PANEL) * PANEL, pe = std::min(n, p0 + PANEL);
    k_potrf_diag<<<1, 256, 0, s>>>(A, n, k0, nbk, dinv + (i64)k * NB * NB, flag);
    if (mr > 0) {
      const i64 tot = (i64)mr * nbk;
      k_copy2d<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(A + (i64)r0 * n + k0, n, panel, NB, mr, nbk);
      if (launch_gemm_stage(F64, st[2 * k], s) != hipSuccess) return GPFVM_E_HIP;
      if (r0 < pe && launch_gemm_stage(F64, st[2 * k + 1], s) != hipSuccess) return GPFVM_E_HIP;
    }
    if (r0 == pe && pe < n &&          // the panel is done: the trailing matrix takes its update
        syrk_rows_lower_sub(n - pe, pe - p0, A + (i64)pe * n + p0, n, A + (i64)pe * n + pe, n, s) != hipSuccess) {
      err = "Cholesky trailing update failed";
      return GPFVM_E_HIP;
    }
  }
  int hflag = 0;
  if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return GPFVM_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return GPFVM_E_HIP;
  if (hflag != 0) {
    err = "point-observation Gram block is not positive definite (Cholesky pivot <= 0 in block at row " +
          std::to_string(hflag - 1) + ")";
    return GPFVM_E_NOTPD;
  }
  {
    const i64 tot = (i64)n * n;
    k_zero_upper<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(A, n, n);
  }
  if (!Linv) return GPFVM_OK;

  // Triangular inverse X = L^{-1}, recursively: with L split at a block boundary
  // into [[L11, 0], [L21, L22]], X11 = L11^{-1} and X22 = L22^{-1} come from the
  // halves and X21 = -X22 (L21 X11), refined once with the residual of the block
  // row, X21 -= X22 (L22 X21 + L21 X11).  The refinement keeps the residual
  // L X - I at the level of the column-by-column substitution (without it,
  // |L X - I| grows from 7e-13 to 5e-10 on a point block of condition 1e9).  The
  // solver's corrected triangular solves would tolerate that, but the posterior
  // variance sf2 - ||L^{-1} k||^2 cancels where it is small: without the refinement
  // the wave problem's variance after 30 iterations moves 1.2e-6 from the oracle's,
  // beyond the 1e-6 it meets with it.  The 64 x 64 leaves are the
  // inverses the diagonal factorisation wrote to dinv; every product is a library
  // TRMM (out of place, through two workspaces of the largest L21), so the work
  // is in products as large as the matrix allows.
  if (hipMemsetAsync(Linv, 0, (size_t)n * n * sizeof(double), s) != hipSuccess) return GPFVM_E_HIP;
  for (int i = 0; i < nblk; ++i) {
    const int i0 = i * NB, nbi = std::min(NB, n - i0);
    k_copy2d<<<(unsigned)(((i64)nbi * nbi + 255) / 256), 256, 0, s>>>(dinv + (i64)i * NB * NB, NB,
                                                                         Linv + (i64)i0 * n + i0, n, nbi, nbi);
  }
  if (nblk < 2) return hipStreamSynchronize(s) == hipSuccess ? GPFVM_OK : GPFVM_E_HIP;
  Arena work;                          // the workspaces go back to the cache afterwards
  work.cache = arena.cache;
  const int top1 = (nblk / 2) * NB;
  const size_t wbytes = (size_t)top1 * (n - top1) * sizeof(double);
  double* W = (double*)work.alloc(wbytes);
  double* R = (double*)work.alloc(wbytes);
  if (!W || !R) { work.release(); err = "out of device memory (inverse workspace)"; return GPFVM_E_NOMEM; }
  std::function<hipError_t(int, int)> inv = [&](int b0, int nbk) -> hipError_t {
    if (nbk <= 1) return hipSuccess;
    const int h1 = nbk / 2;
    hipError_t e = inv(b0, h1);
    if (e == hipSuccess) e = inv(b0 + h1, nbk - h1);
    if (e != hipSuccess) return e;
    const int o = b0 * NB, n1 = h1 * NB, n2 = std::min(n, (b0 + nbk) * NB) - o - n1;
    const i64 m = (i64)n2 * n1;
    const double* X11 = Linv + (i64)o * n + o;
    const double* X22 = Linv + (i64)(o + n1) * n + o + n1;
    const double* L21 = A + (i64)(o + n1) * n + o;
    const double* L22 = A + (i64)(o + n1) * n + o + n1;
    double* X21 = Linv + (i64)(o + n1) * n + o;
    // W = L21 X11 ; X21 = -X22 W ; R = L22 X21 + W ; W = X22 R ; X21 -= W
    if ((e = trmm_rows_right_lower(n2, n1, 1.0, X11, n, L21, n, W, n1, s)) != hipSuccess) return e;
    if ((e = trmm_rows_left_lower(n2, n1, -1.0, X22, n, W, n1, X21, n, s)) != hipSuccess) return e;
    if ((e = trmm_rows_left_lower(n2, n1, 1.0, L22, n, X21, n, R, n1, s)) != hipSuccess) return e;
    if ((e = launch_axpby(m, 1.0, W, 1.0, R, s)) != hipSuccess) return e;
    if ((e = trmm_rows_left_lower(n2, n1, 1.0, X22, n, R, n1, W, n1, s)) != hipSuccess) return e;
    k_axpy2d<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(W, n1, X21, n, n2, n1, -1.0);
    return hipGetLastError();
  };
  // With n = 64 * 2^l the tree is balanced: the nodes of one level have equal sizes and
  // equal strides, and each level runs as six batched launches instead of six per node.
  auto levels = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (int sz = 2; sz <= nblk && e == hipSuccess; sz *= 2) {
      const int count = nblk / sz, n1 = sz / 2 * NB, n2 = n1;
      const i64 m = (i64)n2 * n1, nodes = (i64)sz * NB * (n + 1), ws = m;   // node stride on the diagonal
      const double* X11 = Linv;
      const double* X22 = Linv + (i64)n1 * (n + 1);
      const double* L21 = A + (i64)n1 * n;
      const double* L22 = A + (i64)n1 * (n + 1);
      double* X21 = Linv + (i64)n1 * n;
      if ((e = trmm_rows_right_lower(n2, n1, 1.0, X11, n, L21, n, W, n1, s, count, nodes, nodes, ws)) != hipSuccess ||
          (e = trmm_rows_left_lower(n2, n1, -1.0, X22, n, W, n1, X21, n, s, count, nodes, ws, nodes)) != hipSuccess ||
          (e = trmm_rows_left_lower(n2, n1, 1.0, L22, n, X21, n, R, n1, s, count, nodes, nodes, ws)) != hipSuccess ||
          (e = launch_axpby(m * count, 1.0, W, 1.0, R, s)) != hipSuccess ||
          (e = trmm_rows_left_lower(n2, n1, 1.0, X22, n, R, n1, W, n1, s, count, nodes, ws, ws)) != hipSuccess)
        return e;
      k_axpy2d<<<dim3((unsigned)((m + 255) / 256), (unsigned)count), 256, 0, s>>>(W, n1, X21, n, n2, n1, -1.0, ws, nodes);
      e = hipGetLastError();
    }
    return e;
  };
  const bool balanced = (n % NB == 0) && ((nblk & (nblk - 1)) == 0);
  const hipError_t ie = balanced ? levels() : inv(0, nblk);
  const hipError_t se = hipStreamSynchronize(s);
  work.release();
  if (ie != hipSuccess || se != hipSuccess) { err = "triangular inverse failed"; return GPFVM_E_HIP; }
  return GPFVM_OK;
}

}  // namespace gpfvm
