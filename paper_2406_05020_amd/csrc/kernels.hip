// Device kernels of the gpfvm library: closed-form 1-D factors, the grouped
// MFMA GEMM that carries every Kronecker mode product, and small BLAS-1 /
// elementwise kernels.
#include <hip/hip_runtime.h>

#include "common.h"
#include "reduce.h"
#include <type_traits>

namespace gpfvm {

// ============================================================================
// 1-D squared-exponential calculus (Sec. 3.1 eq. linop-simplified)
//
// With k(r) = exp(-r^2 / (2 l^2)), u = r / l:
//   k^(m)(r)  = (-1/l)^m He_m(u) k(r)                      m >= 0
//   k^(-1)(r) = l sqrt(pi/2) erf(u / sqrt 2)               (antiderivative)
//   k^(-2)(r) = l sqrt(pi/2) r erf(u / sqrt 2) + l^2 (k(r) - 1)
// (He_m: probabilists' Hermite polynomials, He_{n+1} = u He_n - n He_{n-1};
// the constant -l^2 in k^(-2) is immaterial below and keeps the values small.)
// By the fundamental theorem of calculus applied to both cell integrals,
//   int_I int_I' d^p_s d^q_s' k(s - s')  = (-1)^q  D2[k^(p+q-2)](I, I')
//   D2[g](I, I') = g(b - a') - g(a - a') - g(b - b') + g(a - b')
//   int_I' d^p_x d^q_s' k(x - s')        = (-1)^q (k^(p+q-1)(x - a') - k^(p+q-1)(x - b'))
//   d^p_x d^q_x' k(x - x')               = (-1)^q k^(p+q)(x - x')
// ============================================================================
__device__ __forceinline__ double se_deriv(int m, double r, double ell) {
  const double u = r / ell;
  const double e = exp(-0.5 * u * u);
  if (m == -2) {
    const double c = ell * 1.2533141373155002512;   // l sqrt(pi/2)
    return c * r * erf(u * 0.70710678118654752440) + ell * ell * expm1(-0.5 * u * u);
  }
  if (m == -1) return ell * 1.2533141373155002512 * erf(u * 0.70710678118654752440);
  double h0 = 1.0, h1 = u;
  double hm = (m == 0) ? h0 : h1;
  for (int k = 1; k < m; ++k) {
    const double h2 = u * h1 - k * h0;
    h0 = h1;
    h1 = h2;
    hm = h2;
  }
  double s = 1.0;
  const double il = -1.0 / ell;
  for (int k = 0; k < m; ++k) s *= il;
  return s * hm * e;
}

// ============================================================================
// Half-integer Matern kernels (Sec. 3.1): nu = q + 1/2, q = 0..3,
//   k(r) = e^{-s} p_q(s),  s = c |r| / l,  c = sqrt(2q + 1),
//   p_0 = 1, p_1 = 1 + s, p_2 = 1 + s + s^2/3, p_3 = 1 + s + 2s^2/5 + s^3/15.
// Derivatives and antiderivatives stay exponential times polynomial:
//   k^(m)(r)  = sgn(r)^m (c/l)^m e^{-s} P_m(s),   P_0 = p_q, P_{j+1} = d/ds P_j - P_j,
//   k^(-1)(r) = sgn(r) (l/c) (A1 - e^{-s} Q1(s)), Q1 = sum_j d^j/ds^j p_q, A1 = Q1(0),
//   k^(-2)(r) = (l/c)^2 (A1 s - A2 + e^{-s} Q2(s)), Q2 = sum_j d^j/ds^j Q1, A2 = Q2(0),
// because d/ds [-e^{-s} sum_j d^j/ds^j Q] = e^{-s} Q.  k^(-2) is evaluated as
// A1 s + A2 expm1(-s) + e^{-s} (Q2(s) - A2) to keep its O(s^2) size near 0.
// ============================================================================
__device__ __forceinline__ double poly3(const double* a, double s) {
  return ((a[3] * s + a[2]) * s + a[1]) * s + a[0];
}

// b = sum_j d^j/ds^j a for a cubic a (coefficients, lowest first)
__device__ __forceinline__ void sum_of_derivatives(const double* a, double* b) {
  b[3] = a[3];
  b[2] = a[2] + 3.0 * a[3];
  b[1] = a[1] + 2.0 * a[2] + 6.0 * a[3];
  b[0] = a[0] + a[1] + 2.0 * a[2] + 6.0 * a[3];
}

__device__ double matern_deriv(int q, int m, double r, double ell) {
  double P[4] = {1.0, 0.0, 0.0, 0.0};
  if (q >= 1) P[1] = 1.0;
  if (q == 2) P[2] = 1.0 / 3.0;
  if (q == 3) { P[2] = 0.4; P[3] = 1.0 / 15.0; }
  const double c = sqrt(2.0 * q + 1.0);
  const double s = c * fabs(r) / ell;
  const double e = exp(-s);
  const double sg = (r > 0.0) ? 1.0 : (r < 0.0 ? -1.0 : 0.0);
  if (m >= 0) {
    double f = 1.0;
    for (int j = 0; j < m; ++j) {       // P <- d/ds P - P
      P[0] = P[1] - P[0];
      P[1] = 2.0 * P[2] - P[1];
      P[2] = 3.0 * P[3] - P[2];
      P[3] = -P[3];
      f *= c / ell;
    }
    const double v = f * e * poly3(P, s);
    return (m & 1) ? sg * v : v;
  }
  double Q1[4], Q2[4];
  sum_of_derivatives(P, Q1);
  const double A1 = Q1[0];
  if (m == -1) return sg * (ell / c) * (A1 - e * poly3(Q1, s));
  sum_of_derivatives(Q1, Q2);
  const double A2 = Q2[0];
  const double tail = s * ((Q2[3] * s + Q2[2]) * s + Q2[1]);
  const double lc = ell / c;
  return lc * lc * (A1 * s + A2 * expm1(-s) + e * tail);
}

// kq < 0: squared exponential; kq = 0..3: Matern nu = kq + 1/2.
__device__ __forceinline__ double kernel_deriv(int kq, int m, double r, double ell) {
  return kq < 0 ? se_deriv(m, r, ell) : matern_deriv(kq, m, r, ell);
}

// kind 0: cell-cell; a1, a2 are edge arrays (n1+1, n2+1).
// kind 1: point-cell; a1 points (n1), a2 edges (n2+1).
// kind 2: point-point; a1 (n1), a2 (n2) points.
__global__ void k_factor(int kind, int kq, int p, int q, int n1, const double* __restrict__ a1, int n2,
                         const double* __restrict__ a2, double ell, double scale,
                         double* __restrict__ out, i64 ld) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (i64)n1 * n2) return;
  const int i = (int)(idx / n2), j = (int)(idx % n2);
  const double sgn = (q & 1) ? -scale : scale;
  double v;
  if (kind == 0) {
    const double a = a1[i], b = a1[i + 1], c = a2[j], d = a2[j + 1];
    const int m = p + q - 2;
    v = (kernel_deriv(kq, m, b - c, ell) - kernel_deriv(kq, m, a - c, ell)) -
        (kernel_deriv(kq, m, b - d, ell) - kernel_deriv(kq, m, a - d, ell));
  } else if (kind == 1) {
    const double x = a1[i];
    const int m = p + q - 1;
    v = kernel_deriv(kq, m, x - a2[j], ell) - kernel_deriv(kq, m, x - a2[j + 1], ell);
  } else {
    v = kernel_deriv(kq, p + q, a1[i] - a2[j], ell);
  }
  out[(i64)i * ld + j] = sgn * v;
}

hipError_t launch_factor(int kind, int kq, int p, int q, int n1, const double* a1, int n2, const double* a2,
                         double ell, double scale, double* out, i64 ld, hipStream_t s) {
  const i64 tot = (i64)n1 * n2;
  if (tot == 0) return hipSuccess;
  const int bs = 256;
  k_factor<<<dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s>>>(kind, kq, p, q, n1, a1, n2, a2, ell,
                                                                      scale, out, ld);
  return hipGetLastError();
}

// ============================================================================
// Grouped GEMM on MFMA (descriptor semantics in common.h).  Two kernels share
// the descriptor format: an LDS-tiled one for stages with many output tiles
// and short K, and a split-K one for long reductions over few tiles.
// Lane layout of the 16x16x4 MFMA (f64 and f32): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator register i of lane l
// holds D[row][l % 16] with row = 4 * (l / 16) + i for f32 but
// row = l / 16 + 4 * i for f64 (both checked on gfx950 by a lane probe).
// ============================================================================
template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct MfmaOp<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// ----------------------------------------------------------------------------
// Split-K variant: four wavefronts share one 32x32 output tile and split its K
// range in chunks of 16 (wave w takes chunks w, w+4, ...).  Operands go from
// global memory (L2-resident for these sizes) straight into MFMA registers in
// the lane layout above, with the next chunk's loads issued before the current
// chunk's MFMAs; no LDS staging and no barriers in the K loop.  The four
// partial accumulators are summed through LDS at the end.  Built for the
// latency-bound shapes of the hot path: few output tiles, long K.
// ----------------------------------------------------------------------------
constexpr int SK_WAVES = 4;
constexpr int SK_CHUNK = 16;

template <typename T>
struct Chunk {
  T a[4][2], b[4][2];   // [k-step][block]
};

template <typename T>
__device__ __forceinline__ void sk_load(Chunk<T>& c, const T* __restrict__ A, const T* __restrict__ B, const Seg& S,
                                        int m0, int n0, int M, int N, int k0, int kbeg, int kend, int lr, int lk,
                                        T alpha) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = k0 + 4 * kk + lk;
    const bool kin = (k >= kbeg) && (k < kend);
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int row = m0 + blk * 16 + lr;
      const int col = n0 + blk * 16 + lr;
      c.a[kk][blk] = (kin && row < M) ? alpha * A[(i64)row * S.a_rs + (i64)k * S.a_cs] : (T)0;
      c.b[kk][blk] = (kin && col < N) ? B[(i64)k * S.b_rs + (i64)col * S.b_cs] : (T)0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(64 * SK_WAVES) void k_gemm_sk(const GemmDesc* __restrict__ descs, int ndesc) {
  typedef typename MfmaOp<T>::v4 v4;
  __shared__ T red[SK_WAVES - 1][16][64];

  const i64 tile = blockIdx.x;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& D = descs[lo];
  const i64 local = tile - D.tile_begin;
  const int tn = (int)(local % D.tiles_n);
  const i64 rest = local / D.tiles_n;
  const int tm = (int)(rest % D.tiles_m);
  const i64 b = rest / D.tiles_m;
  if (b >= D.batch) return;
  if (D.lower_only && tn > tm) return;
  const int m0 = tm * TILE, n0 = tn * TILE;
  const int M = D.M, N = D.N;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;

  v4 acc[2][2][2];   // [slot][bm][bn]
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[s][i][j][r] = 0;
  bool used1 = false;

  for (int g = 0; g < D.nseg; ++g) {
    const Seg& S = D.seg[g];
    const T* __restrict__ A = reinterpret_cast<const T*>(S.A) + b * S.a_bs;
    const T* __restrict__ B = reinterpret_cast<const T*>(S.B) + b * S.b_bs;
    const T alpha = (T)S.alpha;
    int kbeg = 0, kend = S.K;
    if (S.tri == 1) kend = min(S.K, m0 + TILE);
    else if (S.tri == 2) kbeg = m0;
    else if (S.tri == 3) kend = min(S.K, n0 + TILE);
    else if (S.tri == 4) kbeg = n0;
    if (S.slot) used1 = true;
    const int first = kbeg + SK_CHUNK * wave;
    if (first >= kend) continue;
    Chunk<T> cur, nxt;
    sk_load(cur, A, B, S, m0, n0, M, N, first, kbeg, kend, lr, lk, alpha);
    for (int k0 = first; k0 < kend; k0 += SK_CHUNK * SK_WAVES) {
      const int kn = k0 + SK_CHUNK * SK_WAVES;
      if (kn < kend) sk_load(nxt, A, B, S, m0, n0, M, N, kn, kbeg, kend, lr, lk, alpha);
      if (S.slot == 0) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          acc[0][0][0] = MfmaOp<T>::mac(cur.a[kk][0], cur.b[kk][0], acc[0][0][0]);
          acc[0][0][1] = MfmaOp<T>::mac(cur.a[kk][0], cur.b[kk][1], acc[0][0][1]);
          acc[0][1][0] = MfmaOp<T>::mac(cur.a[kk][1], cur.b[kk][0], acc[0][1][0]);
          acc[0][1][1] = MfmaOp<T>::mac(cur.a[kk][1], cur.b[kk][1], acc[0][1][1]);
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          acc[1][0][0] = MfmaOp<T>::mac(cur.a[kk][0], cur.b[kk][0], acc[1][0][0]);
          acc[1][0][1] = MfmaOp<T>::mac(cur.a[kk][0], cur.b[kk][1], acc[1][0][1]);
          acc[1][1][0] = MfmaOp<T>::mac(cur.a[kk][1], cur.b[kk][0], acc[1][1][0]);
          acc[1][1][1] = MfmaOp<T>::mac(cur.a[kk][1], cur.b[kk][1], acc[1][1][1]);
        }
      }
      cur = nxt;
    }
  }

  // cross-wave reduction, one slot at a time
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s == 1 && !used1) break;
    if (wave > 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wave - 1][(i * 2 + j) * 4 + r][lane] = acc[s][i][j][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int w = 0; w < SK_WAVES - 1; ++w)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[s][i][j][r] += red[w][(i * 2 + j) * 4 + r][lane];
    }
    __syncthreads();
  }
  if (wave != 0) return;

  T* __restrict__ C = reinterpret_cast<T*>(D.C) + b * D.c_bs;
  const T* __restrict__ X = D.X ? reinterpret_cast<const T*>(D.X) + b * D.x_bs : nullptr;
  const double* __restrict__ E = D.escale ? D.escale + b * D.e_bs : nullptr;
  const T beta = (T)D.beta, gamma = (T)D.gamma;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + bm * 16 + MfmaOp<T>::row(lk, r);
        const int col = n0 + bn * 16 + lr;
        if (row < M && col < N && !(D.lower_only && col > row)) {
          T v = acc[0][bm][bn][r];
          if (used1 && E) v += (T)E[(i64)row * D.e_rs + (i64)col * D.e_cs] * acc[1][bm][bn][r];
          if (X) v += gamma * X[(i64)row * D.x_rs + (i64)col * D.x_cs];
          T* cp = C + (i64)row * D.c_rs + (i64)col * D.c_cs;
          if (beta != (T)0) v += beta * *cp;
          *cp = v;
        }
      }
}

// ----------------------------------------------------------------------------
// LDS-tiled variant.  A workgroup owns a BM x BN output tile; its wavefronts
// form KS groups, each with one wavefront per 16x16 block of the tile.  K
// advances in chunks of 16 KS: the threads load the next chunk of both
// operands into registers (coalesced along whichever index is contiguous)
// while group g runs the MFMAs of k-rows [16 g, 16 g + 16) of the current
// chunk from the other half of a double-buffered LDS tile; one barrier per
// chunk.  With KS > 1 the groups' partial accumulators are summed through LDS
// in a fixed order at the end (fewer sequential chunks for short, latency-
// bound stages).  Triangular segments restrict the chunk range to the blocks
// that can be nonzero for this tile (the zero triangle must hold zeros), and
// lower_only skips tiles above the diagonal (BM == BN).
// ----------------------------------------------------------------------------
// One workgroup of NT threads: out[row] = M[row,:] . x (/ eta[row]), summed in
// a fixed order (two interleaved accumulators per thread, then a wavefront
// tree, then the wavefronts in order).  red: NT / 64 doubles of LDS.
// Operand pointers read from a descriptor are generic; as global-address-space
// pointers (the same address for device allocations) their loads become
// global loads, whose completion counter is in order, so a load can stay in
// flight across the LDS stores of an earlier chunk.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> to_global(const T* p) {
  return (gptr<T>)p;
}

// Dot product of q[c_lo, c_hi) and x[c_lo, c_hi) by one workgroup of NT
// threads, valid in thread 0.  Each thread issues RD_U loads of both vectors
// before it multiplies; the sum runs in a fixed order (RD_U accumulators per
// thread, a pairwise tree over them, a wavefront tree, then the wavefronts in
// order).  red: NT / 64 doubles of LDS.
constexpr int RD_U = 16;

template <int NT>
__device__ __forceinline__ double dot_range(const double* __restrict__ q, const double* __restrict__ x, i64 c_lo,
                                            i64 c_hi, double* red, const double* __restrict__ xm = nullptr) {
  double acc[RD_U];
#pragma unroll
  for (int u = 0; u < RD_U; ++u) acc[u] = 0.0;
  for (i64 c0 = c_lo + threadIdx.x; c0 < c_hi; c0 += (i64)NT * RD_U) {
    double qv[RD_U], xv[RD_U];
#pragma unroll
    for (int u = 0; u < RD_U; ++u) {
      const i64 c = c0 + (i64)u * NT;
      qv[u] = c < c_hi ? q[c] : 0.0;
      xv[u] = c < c_hi ? x[c] : 0.0;
    }
    if (xm) {
#pragma unroll
      for (int u = 0; u < RD_U; ++u) {
        const i64 c = c0 + (i64)u * NT;
        xv[u] -= c < c_hi ? xm[c] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < RD_U; ++u) acc[u] = fma(qv[u], xv[u], acc[u]);
  }
#pragma unroll
  for (int w = RD_U / 2; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
  double v = acc[0];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// One workgroup of NT threads: out[row] = M[row,:] . x (/ eta[row]).
template <int NT>
__device__ __forceinline__ void rows_dot_block(i64 N, const double* __restrict__ M, const double* __restrict__ x,
                                               const double* __restrict__ eta, double* __restrict__ out, int row,
                                               double* red) {
  const double s = dot_range<NT>(M + (i64)row * N, x, 0, N, red);
  if (threadIdx.x == 0) out[row] = eta ? s / eta[row] : s;
}

// One workgroup of NT threads: out[c] = sum_j M[j][c] v[j] for the 64
// columns c of block `blk`.  The sum runs in the order of k_cols_update:
// 16 partial sums, partial w over the rows j = w, w + 16, ... in turn, then
// the partials in order (each wavefront keeps 16 / (NT / 64) of them).
// red: 1024 doubles of LDS.
constexpr int CS_PARTS = 16;

template <int NT>
__device__ __forceinline__ void cols_sum_block(int nr, i64 N, const double* __restrict__ M,
                                               const double* __restrict__ v, double* __restrict__ out, i64 blk,
                                               double* red) {
  constexpr int NW = NT / 64, PER = CS_PARTS / NW;
  static_assert(PER * NW == CS_PARTS, "partial sums per wavefront");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const i64 c = blk * 64 + lane;
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;
  if (c < N) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int w = wave + k * NW;
#pragma unroll 4
      for (int j = w; j < nr; j += CS_PARTS) acc[k] = fma(M[(i64)j * N + c], v[j], acc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) red[(wave + k * NW) * 64 + lane] = acc[k];
  __syncthreads();
  if (wave == 0 && c < N) {
    double t = 0.0;
    for (int w = 0; w < CS_PARTS; ++w) t += red[w * 64 + lane];
    out[c] = t;
  }
}

__global__ __launch_bounds__(512) void k_cols_sum(int nr, i64 N, const double* __restrict__ M,
                                                  const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[64 * CS_PARTS];
  cols_sum_block<512>(nr, N, M, v, out, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// Factored point correction (QFactor), one workgroup of NT threads each.
//
// qf_v_block: work unit u = QF_UW consecutive free indices j of one piece r.
// It forms w_r[j] (x contracted with q_r over the pinned dimension) for those
// j: pinned dimension 0 with the unit's columns across QF_UW lanes and the
// rows split into NT / QF_UW interleaved phases (their partial sums then added
// in order), pinned dimension 1 with a wavefront per row.  Then it writes the
// unit's share of v = P w for every a < W, sum_k P[b_k][a] w[b_k] (P is
// symmetric, so rows of P are read contiguously), stored piece-major: output
// a = off_r + j of piece r goes to vpart[nunit off_r + u nf_r + j].  Narrow
// units keep every phase to about one round of loads.  wl: NT + QF_UW doubles.
// ---------------------------------------------------------------------------
constexpr int QF_U = 4;

template <int NT>
__device__ void qf_v_block(const QFactor& F, const double* __restrict__ x, double* __restrict__ vpart, int u,
                           double* wl) {
  constexpr int NW = NT / 64, NPH = NT / QF_UW;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n0 = F.n0, n1 = F.n1, W = F.W;
  int r = 0, j0 = 0;
  for (int uu = u; r < F.R; ++r) {
    const int cnt = ((F.p[r] == 0 ? n1 : n0) + QF_UW - 1) / QF_UW;
    if (uu < cnt) { j0 = uu * QF_UW; break; }
    uu -= cnt;
  }
  const int p = F.p[r], nf = p == 0 ? n1 : n0;
  const int jn = min(QF_UW, nf - j0);
  const double* __restrict__ q = F.q[r];
  const double* __restrict__ P = F.P;
  const int b0 = F.off[r] + j0;
  double* part = wl;
  double* wc = wl + NT;
  // the first QF_PF of this thread's P entries for output a = tid, loaded before w is
  // formed (more would raise the kernel's register count above that of its GEMM tiles)
  constexpr int QF_PF = 8;
  double pr[QF_PF];
#pragma unroll
  for (int k = 0; k < QF_PF; ++k) pr[k] = (tid < W && k < jn) ? P[(i64)(b0 + k) * W + tid] : 0.0;
  if (p == 0) {
    const int k = tid % QF_UW, ph = tid / QF_UW;
    double acc = 0.0;
    if (k < jn) {
      const int c = j0 + k;
      for (int i0 = ph; i0 < n0; i0 += NPH * QF_U) {
        double xv[QF_U], qv[QF_U];
#pragma unroll
        for (int m = 0; m < QF_U; ++m) {
          const int i = i0 + m * NPH;
          xv[m] = i < n0 ? x[(i64)i * n1 + c] : 0.0;
          qv[m] = i < n0 ? q[i] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < QF_U; ++m) acc = fma(qv[m], xv[m], acc);
      }
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < QF_UW) {
      double t = 0.0;
      for (int h = 0; h < NPH; ++h) t += part[h * QF_UW + tid];
      wc[tid] = t;
    }
  } else {
    for (int k = wave; k < jn; k += NW) {
      const int i = j0 + k;
      double t = 0.0;
      for (int c = lane; c < n1; c += 64) t = fma(q[c], x[(i64)i * n1 + c], t);
      for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
      if (lane == 0) wc[k] = t;
    }
  }
  __syncthreads();
  for (int a = tid; a < W; a += NT) {
    double t = 0.0;
    if (a == tid) {
#pragma unroll
      for (int k = 0; k < QF_PF; ++k)
        if (k < jn) t = fma(pr[k], wc[k], t);
      for (int k = QF_PF; k < jn; ++k) t = fma(P[(i64)(b0 + k) * W + a], wc[k], t);
    } else {
#pragma unroll 16
      for (int k = 0; k < jn; ++k) t = fma(P[(i64)(b0 + k) * W + a], wc[k], t);
    }
    // pieces pinned in dimension 0 hold [0, w0) in blocks of n1, the others blocks of n0
    const int nfa = a < F.w0 ? n1 : n0;
    const int j = a < F.w0 ? a % n1 : (a - F.w0) % n0;
    vpart[(i64)F.nunit * (a - j) + (i64)u * nfa + j] = t;
  }
}

constexpr int QF_THREADS = 512;

__global__ __launch_bounds__(QF_THREADS) void k_qf_v(const QFactor* __restrict__ F, const double* __restrict__ x,
                                                     double* __restrict__ vpart) {
  __shared__ double wl[QF_THREADS + QF_UW];
  qf_v_block<QF_THREADS>(*F, x, vpart, blockIdx.x, wl);
}

hipError_t launch_qf_v(const QFactor* F, int nunit, const double* x, double* vpart, hipStream_t s) {
  if (nunit < 1) return hipErrorInvalidValue;
  k_qf_v<<<dim3((unsigned)nunit), dim3(QF_THREADS), 0, s>>>(F, x, vpart);
  return hipGetLastError();
}

constexpr int GEMM_KDEPTH1 = 1;

// Wavefront-uniform copies of values read from LDS (equal in every lane), so
// that they live in scalar registers and steer scalar control flow.
__device__ __forceinline__ int ufl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ i64 ufl(i64 x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return (i64)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double ufl(double x) { return __longlong_as_double(ufl((i64)__double_as_longlong(x))); }
template <typename P>
__device__ __forceinline__ P* ufl(P* p) {
  return reinterpret_cast<P*>((uintptr_t)ufl((i64)(uintptr_t)p));
}

template <typename T>
using gptrw = __attribute__((address_space(1))) T*;

// Workgroups are dispatched to the 8 XCDs in turn (workgroup w runs on XCD
// w % 8), and each XCD has its own L2.  Tiles are dealt to the XCDs in chunks
// of GEMM_XCHUNK consecutive tiles (a batch slab of 2 x 2 tiles, or tiles
// sharing an operand row block), so that a chunk is fetched into one L2, and
// chunk c goes to XCD c % 8, so that every XCD gets an even share of
// triangular stages whose tiles' K ranges grow with the row block.  A
// bijection of [0, n); the last n mod (8 GEMM_XCHUNK) tiles keep their order.
constexpr int GEMM_NXCD = 8, GEMM_XCHUNK = 4;

__device__ __forceinline__ i64 xcd_tile(i64 w, i64 n) {
  const i64 full = n / (GEMM_NXCD * GEMM_XCHUNK) * (GEMM_NXCD * GEMM_XCHUNK);
  if (w >= full) return w;
  const i64 x = w % GEMM_NXCD, j = w / GEMM_NXCD;
  return ((j / GEMM_XCHUNK) * GEMM_NXCD + x) * GEMM_XCHUNK + j % GEMM_XCHUNK;
}

template <typename T, int BM, int BN, int KS, bool SLOT1, bool RIDE>
__global__ __launch_bounds__(4 * BM * BN / 16 * KS) void k_gemm_lds(const GemmDesc* __restrict__ descs, int ndesc,
                                                                    i64 ntiles, Rider rider) {
  typedef typename MfmaOp<T>::v4 v4;
  // K chunk: 16 per K group; a single K group takes GEMM_KDEPTH1 x 16 per chunk
  constexpr int WNN = BN / 16, NBLK = (BM / 16) * (BN / 16), NT = 64 * NBLK * KS,
                LKC = KS == 1 ? 16 * GEMM_KDEPTH1 : 16 * KS;
  constexpr int EA = BM * LKC / NT, EB = LKC * BN / NT;
  static_assert(EA * NT == BM * LKC && EB * NT == LKC * BN, "tile shape");
  constexpr int NS = SLOT1 ? 2 : 1;
  // LDS tiles are stored k-contiguous, A as [m][k] and B as [n][k], with a row stride of LKC + 2
  // elements.  An operand whose global layout runs along m (or n) is stored one row per lane and
  // meets bank conflicts at this stride; an odd stride removes them (measured: zero conflict
  // cycles) but is no faster, as those stores are off the critical path of the chunk loop.
  constexpr int LS = LKC + 2;
  constexpr int SZA = 2 * BM * LS, SZB = 2 * BN * LS;
  static_assert(NS * (KS - 1) * NBLK * 256 <= SZA + SZB, "reduction space");
  __shared__ T sm[SZA + SZB];
  auto As = [&](int buf, int k, int m) -> T& { return sm[(buf * BM + m) * LS + k]; };
  auto Bs = [&](int buf, int k, int n) -> T& { return sm[SZA + (buf * BN + n) * LS + k]; };

  if constexpr (RIDE) {
    const i64 w = blockIdx.x;
    if (w >= ntiles) {                             // a workgroup of the riding product
      __shared__ double rred[64 * CS_PARTS];
      static_assert(SZA + SZB >= NT + QF_UW, "LDS for the factored correction");
      if (rider.kind == RIDE_ROWS)
        rows_dot_block<NT>(rider.N, rider.M, rider.v, rider.eta, rider.out, (int)(w - ntiles), rred);
      else if (rider.kind == RIDE_COLS)
        cols_sum_block<NT>(rider.nr, rider.N, rider.M, rider.v, rider.out, w - ntiles, rred);
      else
        qf_v_block<NT>(*rider.qf, rider.v, rider.out, (int)(w - ntiles), reinterpret_cast<double*>(sm));
      return;
    }
  }
  const i64 tile = xcd_tile(blockIdx.x, ntiles);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  // This tile's descriptor.  In the K-split kernels (short, latency-bound
  // stages) it is staged in LDS: one round of vector loads finds it among the
  // stage's descriptors (each thread tests one range), one more copies it.
  // Read through scalar loads, its fields form a chain of dependent round
  // trips per segment.  The single-group kernel has long K loops per tile and
  // reads it directly (the extra round trips of staging measured slower there).
  const GemmDesc* Dp = nullptr;
  int lo = 0;
  if constexpr (KS == 1) {
    int hi = ndesc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    Dp = descs + lo;
  } else {
    __shared__ GemmDesc sD;
    __shared__ int sLo;
    static_assert(sizeof(GemmDesc) % 8 == 0, "descriptor words");
    if (ndesc > 1) {
      if (ndesc <= NT) {
        if (tid < ndesc) {
          const i64 t0 = descs[tid].tile_begin;
          const i64 t1 = tid + 1 < ndesc ? descs[tid + 1].tile_begin : (i64)0x7fffffffffffffffLL;
          if (t0 <= tile && tile < t1) sLo = tid;
        }
      } else if (tid == 0) {
        int l = 0, h = ndesc - 1;
        while (l < h) {
          const int mid = (l + h + 1) >> 1;
          if (descs[mid].tile_begin <= tile) l = mid; else h = mid - 1;
        }
        sLo = l;
      }
      __syncthreads();
      lo = ufl(sLo);
    }
    constexpr int NW8 = (int)(sizeof(GemmDesc) / 8);
    const unsigned long long* __restrict__ src = reinterpret_cast<const unsigned long long*>(descs + lo);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&sD);
    for (int w = tid; w < NW8; w += NT) dst[w] = src[w];
    __syncthreads();
    Dp = &sD;
  }
  const GemmDesc& D = *Dp;
  const int tiles_n = ufl(D.tiles_n), tiles_m = ufl(D.tiles_m);
  const i64 local = tile - ufl(D.tile_begin);
  const int tn = (int)(local % tiles_n);
  const i64 rest = local / tiles_n;
  const int tm = (int)(rest % tiles_m);
  const i64 b = rest / tiles_m;
  if (b >= ufl(D.batch)) return;
  const int lower_only = ufl(D.lower_only);
  if (lower_only && tn > tm) return;
  const int M = ufl(D.M), N = ufl(D.N), nseg = ufl(D.nseg);
  const int m0 = tm * BM, n0 = tn * BN;
  const int bidx = wave % NBLK, kg = wave / NBLK;
  const int rb = (bidx / WNN) * 16, cb = (bidx % WNN) * 16;

  // two accumulators per slot, alternating over the MFMAs of a chunk, so that
  // consecutive MFMAs of a wavefront do not wait on each other's result; they
  // are added once at the end
  v4 acc[NS], acc2[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] = acc2[q][r] = 0;

  if constexpr (KS == 1) {
    // one K group: each segment runs its own chunk loop (many short chunks per
    // segment, so the exposed first load of a segment matters little)
    for (int g = 0; g < nseg; ++g) {
      const Seg& S = D.seg[g];
      const gptr<T> __restrict__ A = to_global(reinterpret_cast<const T*>(ufl(S.A)) + b * ufl(S.a_bs));
      const gptr<T> __restrict__ B = to_global(reinterpret_cast<const T*>(ufl(S.B)) + b * ufl(S.b_bs));
      const i64 a_rs = ufl(S.a_rs), a_cs = ufl(S.a_cs), b_rs = ufl(S.b_rs), b_cs = ufl(S.b_cs);
      const T alpha = (T)ufl(S.alpha);
      const int K = ufl(S.K), tri = ufl(S.tri);
      int kbeg = 0, kend = K;
      if (tri == 1) kend = min(K, m0 + BM);
      else if (tri == 2) kbeg = m0;
      else if (tri == 3) kend = min(K, n0 + BN);
      else if (tri == 4) kbeg = n0;
      if (kbeg >= kend) continue;                    // uniform over the workgroup
      const bool akf = (a_cs == 1), bnf = (b_cs == 1);
      const int q = SLOT1 ? ufl(S.slot) : 0;
      // two register sets: the load of chunk c + 2 is issued while chunk c is
      // multiplied, so each load has two chunks of work to hide behind.  Every
      // lane loads (from a clamped, in-range address) and out-of-range elements
      // are multiplied by zero when stored to LDS, so the loads form
      // straight-line code and only the older set is waited for.  (For finite
      // operands this is exactly zero; a non-finite value at a clamped address
      // reaches only outputs whose own sums already hold it.)
      T ra0[EA], rb0[EB], ra1[EA], rb1[EB];
      auto gload = [&](T* ra, T* rbv, int kc) {
  #pragma unroll
        for (int u = 0; u < EA; ++u) {
          const int e = tid + NT * u;
          int k, m;
          if (akf) { k = e % LKC; m = e / LKC; } else { m = e % BM; k = e / BM; }
          const int mm = min(m0 + m, M - 1), kk = min(kc + k, kend - 1);
          ra[u] = A[(i64)mm * a_rs + (i64)kk * a_cs];
        }
  #pragma unroll
        for (int u = 0; u < EB; ++u) {
          const int e = tid + NT * u;
          int k, n;
          if (bnf) { n = e % BN; k = e / BN; } else { k = e % LKC; n = e / LKC; }
          const int nn = min(n0 + n, N - 1), kk = min(kc + k, kend - 1);
          rbv[u] = B[(i64)kk * b_rs + (i64)nn * b_cs];
        }
      };
      // the chunk starting at kc goes to LDS buffer buf; out-of-range elements x 0
      auto sstore = [&](const T* ra, const T* rbv, int buf, int kc) {
  #pragma unroll
        for (int u = 0; u < EA; ++u) {
          const int e = tid + NT * u;
          int k, m;
          if (akf) { k = e % LKC; m = e / LKC; } else { m = e % BM; k = e / BM; }
          const T msk = (m0 + m < M && kc + k < kend) ? alpha : (T)0;
          As(buf, k, m) = msk * ra[u];
        }
  #pragma unroll
        for (int u = 0; u < EB; ++u) {
          const int e = tid + NT * u;
          int k, n;
          if (bnf) { n = e % BN; k = e / BN; } else { k = e % LKC; n = e / LKC; }
          const T msk = (n0 + n < N && kc + k < kend) ? (T)1 : (T)0;
          Bs(buf, k, n) = msk * rbv[u];
        }
      };
      auto mult = [&](int buf) {
  #pragma unroll
        for (int kk = 0; kk < LKC; kk += 4) {
          const int k = kk + lk;
          const T av = As(buf, k, rb + lr);
          const T bv = Bs(buf, k, cb + lr);
          v4* a = ((kk >> 2) & 1) ? acc2 : acc;
          if (q == 0) a[0] = MfmaOp<T>::mac(av, bv, a[0]);
          else a[NS - 1] = MfmaOp<T>::mac(av, bv, a[NS - 1]);
        }
      };
      const int nch = (kend - kbeg + LKC - 1) / LKC;
      const int klast = kbeg + (nch - 1) * LKC;       // start of the last chunk
      __syncthreads();                               // previous segment's reads of buffer 0 are done
      gload(ra0, rb0, kbeg);
      gload(ra1, rb1, min(kbeg + LKC, klast));
      sstore(ra0, rb0, 0, kbeg);
      __syncthreads();
      // chunk c is in LDS buffer c % 2 and, before that, in register set c % 2;
      // past the last chunk the prefetch re-reads it and is never stored
      for (int c = 0; c < nch; c += 2) {
        gload(ra0, rb0, min(kbeg + (c + 2) * LKC, klast));
        mult(0);
        if (c + 1 < nch) sstore(ra1, rb1, 1, kbeg + (c + 1) * LKC);
        __syncthreads();
        if (c + 1 >= nch) break;
        gload(ra1, rb1, min(kbeg + (c + 3) * LKC, klast));
        mult(1);
        if (c + 2 < nch) sstore(ra0, rb0, 0, kbeg + (c + 2) * LKC);
        __syncthreads();
      }
    }

  } else {
    // The K ranges of all segments form one sequence of LKC-wide chunks; the
    // next chunk (possibly the first of the next segment) is prefetched to
    // registers while the current one is multiplied out of LDS.
    struct Ctx {
      gptr<T> A;
      gptr<T> B;
      i64 a_rs, a_cs, b_rs, b_cs;
      T alpha;
      int kbeg, kend, q;
      bool akf, bnf;
    };
    auto ctx_of = [&](int g, Ctx& c) -> bool {      // false: empty K range
      const Seg& S = D.seg[g];
      c.A = to_global(reinterpret_cast<const T*>(ufl(S.A)) + b * ufl(S.a_bs));
      c.B = to_global(reinterpret_cast<const T*>(ufl(S.B)) + b * ufl(S.b_bs));
      c.a_rs = ufl(S.a_rs); c.a_cs = ufl(S.a_cs); c.b_rs = ufl(S.b_rs); c.b_cs = ufl(S.b_cs);
      c.alpha = (T)ufl(S.alpha);
      const int K = ufl(S.K), tri = ufl(S.tri);
      c.kbeg = 0; c.kend = K;
      if (tri == 1) c.kend = min(K, m0 + BM);
      else if (tri == 2) c.kbeg = m0;
      else if (tri == 3) c.kend = min(K, n0 + BN);
      else if (tri == 4) c.kbeg = n0;
      c.akf = (c.a_cs == 1);
      c.bnf = (c.b_cs == 1);
      c.q = SLOT1 ? ufl(S.slot) : 0;
      return c.kbeg < c.kend;
    };
    T ra[EA], rbv[EB];
    auto gload_to = [&](const Ctx& c, int kc, T* oa, T* ob) {
  #pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + NT * u;
        int k, m;
        if (c.akf) { k = e % LKC; m = e / LKC; } else { m = e % BM; k = e / BM; }
        oa[u] = (m0 + m < M && kc + k < c.kend) ? c.A[(i64)(m0 + m) * c.a_rs + (i64)(kc + k) * c.a_cs] : (T)0;
      }
  #pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = tid + NT * u;
        int k, n;
        if (c.bnf) { n = e % BN; k = e / BN; } else { k = e % LKC; n = e / LKC; }
        ob[u] = (n0 + n < N && kc + k < c.kend) ? c.B[(i64)(kc + k) * c.b_rs + (i64)(n0 + n) * c.b_cs] : (T)0;
      }
    };
    auto sstore_from = [&](const Ctx& c, int buf, const T* ia, const T* ib) {
  #pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + NT * u;
        int k, m;
        if (c.akf) { k = e % LKC; m = e / LKC; } else { m = e % BM; k = e / BM; }
        As(buf, k, m) = c.alpha * ia[u];
      }
  #pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = tid + NT * u;
        int k, n;
        if (c.bnf) { n = e % BN; k = e / BN; } else { k = e % LKC; n = e / LKC; }
        Bs(buf, k, n) = ib[u];
      }
    };
    auto gload = [&](const Ctx& c, int kc) { gload_to(c, kc, ra, rbv); };
    auto sstore = [&](const Ctx& c, int buf) { sstore_from(c, buf, ra, rbv); };
    auto mult = [&](int buf, int q) {
  #pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int k = kg * 16 + kk + lk;
        const T av = As(buf, k, rb + lr);
        const T bv = Bs(buf, k, cb + lr);
        v4* a = ((kk >> 2) & 1) ? acc2 : acc;
        if (q == 0) a[0] = MfmaOp<T>::mac(av, bv, a[0]);
        else a[NS - 1] = MfmaOp<T>::mac(av, bv, a[NS - 1]);
      }
    };
    // At most UPF segments of at most one chunk each (the summing stage of a
    // one-rhs operator): every operand load is issued before the first
    // multiply, so the loads' latencies overlap instead of adding up.  The
    // chunks then alternate between the two LDS buffers; the barrier after
    // each store also orders the multiply two chunks back before the next
    // store into its buffer.
    constexpr int UPF = 4;
    bool upfront = nseg <= UPF;
    for (int g = 0; g < nseg; ++g) upfront = upfront && ufl(D.seg[g].K) <= LKC;
    if (upfront) {
      T ua[UPF][EA], ub[UPF][EB];
      Ctx cs[UPF];
      bool live[UPF];
  #pragma unroll
      for (int g = 0; g < UPF; ++g) live[g] = g < nseg && ctx_of(g, cs[g]);   // uniform
  #pragma unroll
      for (int g = 0; g < UPF; ++g)
        if (live[g]) gload_to(cs[g], cs[g].kbeg, ua[g], ub[g]);
      int buf = 0;
  #pragma unroll
      for (int g = 0; g < UPF; ++g) {
        if (!live[g]) continue;
        sstore_from(cs[g], buf, ua[g], ub[g]);
        __syncthreads();
        mult(buf, cs[g].q);
        buf ^= 1;
      }
    }
    int g = 0;
    Ctx cur;
    if (!upfront)
      while (g < nseg && !ctx_of(g, cur)) ++g;       // uniform over the workgroup
    if (!upfront && g < nseg) {
      int kc = cur.kbeg;
      gload(cur, kc);
      sstore(cur, 0);
      __syncthreads();
      int buf = 0;
      for (;;) {
        Ctx nxt = cur;
        int ng = g, nkc = kc + LKC;
        bool more = true;
        if (nkc >= cur.kend) {
          ng = g + 1;
          while (ng < nseg && !ctx_of(ng, nxt)) ++ng;
          more = ng < nseg;
          if (more) nkc = nxt.kbeg;
        }
        if (more) gload(nxt, nkc);
        mult(buf, cur.q);
        if (more) sstore(nxt, buf ^ 1);
        __syncthreads();
        buf ^= 1;
        if (!more) break;
        cur = nxt;
        g = ng;
        kc = nkc;
      }
    }

  }

#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] += acc2[q][r];

  if (KS > 1) {                                    // sum the K groups in a fixed order
    __syncthreads();
    if (kg > 0) {
#pragma unroll
      for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sm[((((q * (KS - 1)) + kg - 1) * NBLK + bidx) * 4 + r) * 64 + lane] = acc[q][r];
    }
    __syncthreads();
    if (kg > 0) return;
#pragma unroll
    for (int q = 0; q < NS; ++q)
      for (int g2 = 1; g2 < KS; ++g2)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] += sm[((((q * (KS - 1)) + g2 - 1) * NBLK + bidx) * 4 + r) * 64 + lane];
  }

  // the descriptor's output fields as uniform values; every addend of the four
  // outputs of this lane is loaded before the first store (an output reads only
  // its own element of X, escale and C)
  const gptrw<T> C = (gptrw<T>)(reinterpret_cast<T*>(ufl(D.C)) + b * ufl(D.c_bs));
  const T* Xp = reinterpret_cast<const T*>(ufl(D.X));
  const double* Ep = ufl(D.escale);
  const gptr<T> X = Xp ? to_global(Xp + b * ufl(D.x_bs)) : nullptr;
  const gptr<double> E = Ep ? to_global(Ep + b * ufl(D.e_bs)) : nullptr;
  const i64 c_rs = ufl(D.c_rs), c_cs = ufl(D.c_cs), x_rs = ufl(D.x_rs), x_cs = ufl(D.x_cs);
  const i64 e_rs = ufl(D.e_rs), e_cs = ufl(D.e_cs);
  const T beta = (T)ufl(D.beta), gamma = (T)ufl(D.gamma);
  bool ok[4];
  T ev[4], xv[4], cv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + rb + MfmaOp<T>::row(lk, r);
    const int col = n0 + cb + lr;
    ok[r] = row < M && col < N && !(lower_only && col > row);
    ev[r] = (SLOT1 && E && ok[r]) ? (T)E[(i64)row * e_rs + (i64)col * e_cs] : (T)0;
    xv[r] = (X && ok[r]) ? X[(i64)row * x_rs + (i64)col * x_cs] : (T)0;
    cv[r] = (beta != (T)0 && ok[r]) ? C[(i64)row * c_rs + (i64)col * c_cs] : (T)0;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + rb + MfmaOp<T>::row(lk, r);
    const int col = n0 + cb + lr;
    if (ok[r]) {
      T v = acc[0][r];
      if (SLOT1 && E) v += ev[r] * acc[NS - 1][r];
      if (X) v += gamma * xv[r];
      if (beta != (T)0) v += beta * cv[r];
      C[(i64)row * c_rs + (i64)col * c_cs] = v;
    }
  }
}

template <typename T, int BM, int KS>
static void launch_lds(const Stage& st, int nd, hipStream_t s) {
  const dim3 block(4 * BM * BM / 16 * KS);
  if constexpr (std::is_same<T, double>::value) {
    if (st.rider.kind != RIDE_NONE) {              // the stage carries a streaming product
      const i64 extra = st.rider.kind == RIDE_COLS ? (st.rider.N + 63) / 64 : st.rider.nr;
      const dim3 grid((unsigned)(st.tiles + extra));
      if (st.slot1)
        k_gemm_lds<T, BM, BM, KS, true, true><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles, st.rider);
      else
        k_gemm_lds<T, BM, BM, KS, false, true><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles, st.rider);
      return;
    }
  }
  const dim3 grid((unsigned)st.tiles);
  if (st.slot1)
    k_gemm_lds<T, BM, BM, KS, true, false><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles, st.rider);
  else
    k_gemm_lds<T, BM, BM, KS, false, false><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles, st.rider);
}

// Thin products: C[b][m][n] = alpha sum_k A[b][m][k] B[b][k][n] for descriptors with M = 1 or
// N = 1 (one segment, no epilogue), one thread per output element in (batch, m, n) order with n
// fastest; the descriptors' tile_begin are their output offsets (ascending).
constexpr int THIN_U = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_thin(const GemmDesc* __restrict__ descs, int nd, i64 total) {
  const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int lo = 0, hi = nd - 1;                     // last descriptor with tile_begin <= idx
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= idx) lo = mid; else hi = mid - 1;
  }
  const GemmDesc& D = descs[lo];
  i64 r = idx - D.tile_begin;
  const i64 n = r % D.N;
  r /= D.N;
  const i64 m = r % D.M;
  const i64 b = r / D.M;
  const Seg& S = D.seg[0];
  const T* __restrict__ A = (const T*)S.A + b * S.a_bs + m * S.a_rs;
  const T* __restrict__ B = (const T*)S.B + b * S.b_bs + n * S.b_cs;
  // K in steps of THIN_U: the step's loads are issued together, then added in order (the same
  // fmas in the same order as one at a time, with THIN_U loads in flight instead of one)
  const int K = S.K;
  const i64 a_cs = S.a_cs, b_rs = S.b_rs;
  double acc = 0.0;
  int k = 0;
  for (; k + THIN_U <= K; k += THIN_U) {
    double av[THIN_U], bv[THIN_U];
#pragma unroll
    for (int u = 0; u < THIN_U; ++u) {
      av[u] = (double)A[(i64)(k + u) * a_cs];
      bv[u] = (double)B[(i64)(k + u) * b_rs];
    }
#pragma unroll
    for (int u = 0; u < THIN_U; ++u) acc = fma(av[u], bv[u], acc);
  }
  for (; k < K; ++k) acc = fma((double)A[(i64)k * a_cs], (double)B[(i64)k * b_rs], acc);
  ((T*)D.C)[b * D.c_bs + m * D.c_rs + n * D.c_cs] = (T)(S.alpha * acc);
}

static hipError_t launch_thin(Elt elt, const Stage& st, hipStream_t s) {
  if (st.nthin == 0 || st.thin_outputs == 0) return hipSuccess;
  const GemmDesc* d = st.d_descs + (st.descs.size() - st.nthin);
  const unsigned g = (unsigned)((st.thin_outputs + 255) / 256);
  if (elt == F64) k_gemm_thin<double><<<g, 256, 0, s>>>(d, st.nthin, st.thin_outputs);
  else k_gemm_thin<float><<<g, 256, 0, s>>>(d, st.nthin, st.thin_outputs);
  return hipGetLastError();
}

// The tiled products of a stage: its first nd descriptors (the thin ones follow them).
static hipError_t launch_tiled(Elt elt, const Stage& st, int nd, hipStream_t s) {
  if (st.rider.kind != RIDE_NONE && (elt != F64 || st.kind == GEMM_SPLITK || st.tiles == 0 || nd == 0)) {
    // the riding product runs on its own where the stage's kernel cannot carry it
    hipError_t e;
    if (st.rider.kind == RIDE_ROWS) {
      if (st.rider.eta) return hipErrorInvalidValue;  // the stand-alone row dots carry no division
      e = launch_rows_dot_full(st.rider.nr, st.rider.N, st.rider.M, st.rider.v, st.rider.out, s);
    } else if (st.rider.kind == RIDE_QFV) {
      e = launch_qf_v(st.rider.qf, st.rider.nr, st.rider.v, st.rider.out, s);
    } else {
      k_cols_sum<<<dim3((unsigned)((st.rider.N + 63) / 64)), dim3(512), 0, s>>>(st.rider.nr, st.rider.N, st.rider.M,
                                                                                st.rider.v, st.rider.out);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (st.tiles == 0 || nd == 0) return hipSuccess;
    Stage plain;
    plain.d_descs = st.d_descs;
    plain.tiles = st.tiles;
    plain.kind = st.kind;
    plain.slot1 = st.slot1;
    return launch_tiled(elt, plain, nd, s);
  }
  if (st.tiles == 0 || nd == 0) return hipSuccess;
  if (elt == F32B) return launch_gemm_bf16s(st, s);
  if (st.kind == GEMM_LDS64) {
    if (elt == F64) launch_lds<double, 64, 1>(st, nd, s); else launch_lds<float, 64, 1>(st, nd, s);
  } else if (st.kind == GEMM_LDS32) {
    if (elt == F64) launch_lds<double, 32, 4>(st, nd, s); else launch_lds<float, 32, 4>(st, nd, s);
  } else if (st.kind == GEMM_LDS16) {
    if (elt == F64) launch_lds<double, 16, 8>(st, nd, s); else launch_lds<float, 16, 8>(st, nd, s);
  } else if (elt == F64) {
    k_gemm_sk<double><<<dim3((unsigned)st.tiles), dim3(64 * SK_WAVES), 0, s>>>(st.d_descs, nd);
  } else {
    k_gemm_sk<float><<<dim3((unsigned)st.tiles), dim3(64 * SK_WAVES), 0, s>>>(st.d_descs, nd);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_stage(Elt elt, const Stage& st, hipStream_t s) {
  // the thin products, then the stage's tiled products (disjoint outputs)
  hipError_t e = launch_thin(elt, st, s);
  if (e != hipSuccess) return e;
  return launch_tiled(elt, st, (int)st.descs.size() - st.nthin, s);
}

// ============================================================================
// elementwise kernels
// ============================================================================
template <typename T>
__global__ void k_scale(const T* __restrict__ src, i64 src_stride, const T* __restrict__ coef, T* __restrict__ dst,
                        i64 dst_stride, i64 n, int nrhs) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const i64 r = i / n, k = i % n;
  dst[r * dst_stride + k] = coef[k] * src[r * src_stride + k];
}

// dst[r*dst_stride + k] = coef[k] * src[r*src_stride + k], k < n, r < nrhs
hipError_t launch_scale(Elt elt, const void* src, i64 src_stride, const void* coef, void* dst, i64 dst_stride, i64 n,
                        int nrhs, hipStream_t s) {
  const i64 tot = n * nrhs;
  if (tot == 0) return hipSuccess;
  const unsigned g = (unsigned)((tot + 255) / 256);
  if (elt == F64)
    k_scale<double><<<g, 256, 0, s>>>((const double*)src, src_stride, (const double*)coef, (double*)dst, dst_stride,
                                      n, nrhs);
  else
    k_scale<float><<<g, 256, 0, s>>>((const float*)src, src_stride, (const float*)coef, (float*)dst, dst_stride, n,
                                     nrhs);
  return hipGetLastError();
}

__global__ void k_axpby(i64 n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
hipError_t launch_axpby(i64 n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_axpby<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, x, b, y);
  return hipGetLastError();
}

__global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, i64 n) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void k_f2d(const float* __restrict__ x, double* __restrict__ y, i64 n) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
hipError_t launch_copy_f64_to_f32(const double* x, float* y, i64 n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_d2f<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}
hipError_t launch_copy_f32_to_f64(const float* x, double* y, i64 n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_f2d<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

struct LinComb { const double* m[8]; double c[8]; int n; };
__global__ void k_lincomb(LinComb lc, i64 len, double* __restrict__ out) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double v = 0;
  for (int k = 0; k < lc.n; ++k) v += lc.c[k] * lc.m[k][i];
  out[i] = v;
}
hipError_t launch_lincomb(int nmat, const double* const* mats, const double* coefs, i64 len,
                          double* out, hipStream_t s) {
  if (nmat > 8) return hipErrorInvalidValue;
  LinComb lc{};
  lc.n = nmat;
  for (int k = 0; k < nmat; ++k) { lc.m[k] = mats[k]; lc.c[k] = coefs[k]; }
  k_lincomb<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(lc, len, out);
  return hipGetLastError();
}

__global__ void k_fill(double* p, double v, i64 n) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill(double* p, double v, i64 n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

__global__ void k_add_diag(double* A, i64 ld, i64 n0, i64 n, const double* vals) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[(n0 + i) * ld + n0 + i] += vals[i];
}
hipError_t launch_add_diag(double* A, i64 ld, i64 n0, i64 n, const double* vals, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_add_diag<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(A, ld, n0, n, vals);
  return hipGetLastError();
}

// ============================================================================
// Deterministic dot product: fixed per-block partition, fixed tree order.
// ============================================================================
constexpr int DOT_BLOCKS = 512;
constexpr int DOT_THREADS = 256;


static_assert(DOT_BLOCKS == DOT_PARTIALS, "dot partial count");

__global__ __launch_bounds__(DOT_THREADS) void k_dot_partial(i64 n, const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             double* __restrict__ partial, i64 bsv) {
  __shared__ double red[DOT_THREADS / 64];
  x += blockIdx.y * bsv;
  y += blockIdx.y * bsv;
  partial += (i64)blockIdx.y * DOT_BLOCKS;
  double acc = 0;
  for (i64 i = (i64)blockIdx.x * DOT_THREADS + threadIdx.x; i < n; i += (i64)DOT_BLOCKS * DOT_THREADS)
    acc += x[i] * y[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < DOT_THREADS / 64; ++w) t += red[w];
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(DOT_THREADS) void k_dot_final(const double* __restrict__ partial,
                                                           double* __restrict__ out, i64 bso) {
  __shared__ double red[DOT_THREADS / 64];
  partial += (i64)blockIdx.x * DOT_BLOCKS;
  out += blockIdx.x * bso;
  double acc = 0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += DOT_THREADS) acc += partial[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < DOT_THREADS / 64; ++w) t += red[w];
    out[0] = t;
  }
}

// final reduction + stopping test: scal[0] = r.r ; converged if r.r <= tol^2 b.b
// (scal[4] = tol^2, scal[3] = b.b); flag[0] = 3 once flag[1] reaches max_iter.
__global__ __launch_bounds__(DOT_THREADS) void k_dot_final_check(const double* __restrict__ partial,
                                                                 double* __restrict__ scal, int* __restrict__ flag,
                                                                 int max_iter, i64 bss, i64 bsf) {
  __shared__ double red[DOT_THREADS / 64];
  partial += (i64)blockIdx.x * DOT_BLOCKS;
  scal += blockIdx.x * bss;
  flag += blockIdx.x * bsf;
  double acc = 0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += DOT_THREADS) acc += partial[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < DOT_THREADS / 64; ++w) t += red[w];
    if (flag[0] == 0) {
      scal[0] = t;
      if (t <= scal[4] * scal[3]) flag[0] = 1;
      else if (flag[1] >= max_iter) flag[0] = 3;
    }
  }
}

hipError_t launch_dot_check(i64 n, const double* x, double* partial, double* scal, int* flag, int max_iter,
                            hipStream_t s, int batch, const BatchStrides& bs) {
  k_dot_partial<<<dim3(DOT_BLOCKS, batch), DOT_THREADS, 0, s>>>(n, x, x, partial, bs.v);
  k_dot_final_check<<<batch, DOT_THREADS, 0, s>>>(partial, scal, flag, max_iter, bs.scal, bs.flag);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// W = G_bb^{-1} U for a small point block in one workgroup (vectors in LDS):
// t = L^{-1} u ; t += L^{-1} (u - L t) ; w = L^{-T} t ; w += L^{-T} (t - L^T w).
// Every product is evaluated as y[i] = add[i] + alpha sum_k A[k][i] x[k] over a
// row-major matrix A (L^T / L^{-T} for the row products, L / L^{-1} for the
// transposed ones), so consecutive lanes read consecutive addresses; the k
// range is split across the wavefronts and the partial sums meet in LDS.
// ----------------------------------------------------------------------------
constexpr int GS_WAVES = 8;
constexpr int GS_THREADS = 64 * GS_WAVES;

// kmode 0: k <= i contributes (A upper-triangular);  kmode 1: k >= i (A lower)
__device__ void gs_prod(int n, const double* __restrict__ A, const double* x, double* y, double alpha,
                        const double* add, int kmode, double (*part)[SMALL_GINV_MAX]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int per = (n + GS_WAVES - 1) / GS_WAVES;
  const int k0 = wave * per, k1 = min(n, k0 + per);
  for (int i = lane; i < n; i += 64) {
    double acc = 0;
    const int lo = kmode ? max(k0, i) : k0;
    const int hi = kmode ? k1 : min(k1, i + 1);
#pragma unroll 4
    for (int k = lo; k < hi; ++k) acc += A[(i64)k * n + i] * x[k];
    part[wave][i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += GS_THREADS) {
    double acc = 0;
#pragma unroll
    for (int w = 0; w < GS_WAVES; ++w) acc += part[w][i];
    y[i] = (add ? add[i] : 0.0) + alpha * acc;
  }
  __syncthreads();
}

__global__ __launch_bounds__(GS_THREADS) void k_ginv_small(int n, const double* __restrict__ L,
                                                           const double* __restrict__ Li,
                                                           const double* __restrict__ Lt,
                                                           const double* __restrict__ Lit,
                                                           const double* __restrict__ U, double* __restrict__ W) {
  __shared__ double u[SMALL_GINV_MAX], t[SMALL_GINV_MAX], r[SMALL_GINV_MAX], w[SMALL_GINV_MAX];
  __shared__ double part[GS_WAVES][SMALL_GINV_MAX];
  for (int i = threadIdx.x; i < n; i += GS_THREADS) u[i] = U[i];
  __syncthreads();
  gs_prod(n, Lit, u, t, 1.0, nullptr, 0, part);    // t = Li u        (Li lower: A = Li^T upper)
  gs_prod(n, Lt, t, r, -1.0, u, 0, part);          // r = u - L t
  gs_prod(n, Lit, r, t, 1.0, t, 0, part);          // t += Li r
  gs_prod(n, Li, t, w, 1.0, nullptr, 1, part);     // w = Li^T t      (A = Li lower)
  gs_prod(n, L, w, r, -1.0, t, 1, part);           // r = t - L^T w
  gs_prod(n, Li, r, u, 1.0, w, 1, part);           // u = w + Li^T r
  for (int i = threadIdx.x; i < n; i += GS_THREADS) W[i] = u[i];
}

hipError_t launch_ginv_small(int nb, const double* L, const double* Linv, const double* Lt, const double* Linvt,
                             const double* U, double* W, hipStream_t s) {
  if (nb < 1 || nb > SMALL_GINV_MAX) return hipErrorInvalidValue;
  k_ginv_small<<<1, GS_THREADS, 0, s>>>(nb, L, Linv, Lt, Linvt, U, W);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Streaming products with a row-major r x N matrix M (the resident point
// correction Q, the stored IterGP directions D and their images S D).
//
// rows_dot:    out[j] = sum_k M[j][k] x[k]  (divided by eta[j] when given).
//   One 1024-thread workgroup per row streams it contiguously with two
//   independent accumulators; fixed-order wavefront and workgroup reductions.
// cols_update: out[c] = base[c] - sum_j M[j][c] u[j]  (also into out2), and
//   optionally out3[c] = base2[c] - sum_j M2[j][c] u[j] with the same u.
//   A 1024-thread workgroup owns 64 columns; its 16 wavefronts take every
//   16th row (64 contiguous doubles per load), u is staged through LDS in
//   blocks, and the 16 partial sums are added in a fixed order.
// Both are deterministic; base may alias out.
// ----------------------------------------------------------------------------
constexpr int CU_WAVES = 16;
static_assert(CU_WAVES == CS_PARTS, "the riding column sums follow the column update's order");
constexpr int CU_BLK = 2048;
constexpr int CU_PF = 8;        // rows per wavefront loaded before the coefficients are staged (small N)
constexpr i64 CU_FINISH_MIN_N = (i64)1 << 18;   // from here on the coefficients are finished beforehand
constexpr int CU_MAXCH = 16;   // most partial sums per coefficient (rows_dot_chunks <= 16)

// Row dots split over column chunks, so that a few long rows still occupy
// the whole chip: part[row * nch + ch] = M[row, chunk ch] . x[chunk ch], the
// chunks being consecutive ranges of ceil(N / nch) columns.  The consumer
// (k_cols_update) adds the nch partials of a row in order.
constexpr int RP_THREADS = 256;
constexpr i64 ROWS_DOT_TWO_MIN_WG = 512;   // two rows per workgroup only where that leaves this many

// dot_range over pairs: q, x (and xm) 16-byte aligned, c_lo and c_hi even.
// RD2_U 16-byte loads of each vector in flight per thread, then the same
// fixed-order reduction.
constexpr int RD2_U = 8;
template <int NT>
__device__ __forceinline__ double dot_range2(const double* __restrict__ q, const double* __restrict__ x, i64 c_lo,
                                             i64 c_hi, double* red, const double* __restrict__ xm) {
  const double2* __restrict__ q2 = reinterpret_cast<const double2*>(q);
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);
  const double2* __restrict__ m2 = reinterpret_cast<const double2*>(xm);
  const i64 plo = c_lo / 2, phi = c_hi / 2;
  double acc[RD2_U];
#pragma unroll
  for (int u = 0; u < RD2_U; ++u) acc[u] = 0.0;
  for (i64 p0 = plo + threadIdx.x; p0 < phi; p0 += (i64)NT * RD2_U) {
    double2 qv[RD2_U], xv[RD2_U];
#pragma unroll
    for (int u = 0; u < RD2_U; ++u) {
      const i64 p = p0 + (i64)u * NT;
      qv[u] = p < phi ? q2[p] : make_double2(0.0, 0.0);
      xv[u] = p < phi ? x2[p] : make_double2(0.0, 0.0);
    }
    if (xm) {
#pragma unroll
      for (int u = 0; u < RD2_U; ++u) {
        const i64 p = p0 + (i64)u * NT;
        const double2 mv = p < phi ? m2[p] : make_double2(0.0, 0.0);
        xv[u].x -= mv.x;
        xv[u].y -= mv.y;
      }
    }
#pragma unroll
    for (int u = 0; u < RD2_U; ++u) acc[u] = fma(qv[u].y, xv[u].y, fma(qv[u].x, xv[u].x, acc[u]));
  }
#pragma unroll
  for (int w = RD2_U / 2; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
  double v = acc[0];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// dot_range2 for two rows q0, q1 against the same x (and xm), whose loads then serve both rows.
// Each row's sum takes exactly the steps of dot_range2 (the same accumulator per element, the same
// reduction), so the results are the same bits.  Valid in thread 0; red holds 2 NT / 64 values.
template <int NT>
__device__ __forceinline__ void dot_range2_two(const double* __restrict__ q0, const double* __restrict__ q1,
                                               const double* __restrict__ x, i64 c_lo, i64 c_hi, double* red,
                                               const double* __restrict__ xm, double& s0, double& s1) {
  const double2* __restrict__ a2 = reinterpret_cast<const double2*>(q0);
  const double2* __restrict__ b2 = reinterpret_cast<const double2*>(q1);
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);
  const double2* __restrict__ m2 = reinterpret_cast<const double2*>(xm);
  const i64 plo = c_lo / 2, phi = c_hi / 2;
  double acc0[RD2_U], acc1[RD2_U];
#pragma unroll
  for (int u = 0; u < RD2_U; ++u) acc0[u] = acc1[u] = 0.0;
  for (i64 p0 = plo + threadIdx.x; p0 < phi; p0 += (i64)NT * RD2_U) {
    double2 av[RD2_U], bv[RD2_U], xv[RD2_U];
#pragma unroll
    for (int u = 0; u < RD2_U; ++u) {
      const i64 p = p0 + (i64)u * NT;
      av[u] = p < phi ? a2[p] : make_double2(0.0, 0.0);
      bv[u] = p < phi ? b2[p] : make_double2(0.0, 0.0);
      xv[u] = p < phi ? x2[p] : make_double2(0.0, 0.0);
    }
    if (xm) {
#pragma unroll
      for (int u = 0; u < RD2_U; ++u) {
        const i64 p = p0 + (i64)u * NT;
        const double2 mv = p < phi ? m2[p] : make_double2(0.0, 0.0);
        xv[u].x -= mv.x;
        xv[u].y -= mv.y;
      }
    }
#pragma unroll
    for (int u = 0; u < RD2_U; ++u) {
      acc0[u] = fma(av[u].y, xv[u].y, fma(av[u].x, xv[u].x, acc0[u]));
      acc1[u] = fma(bv[u].y, xv[u].y, fma(bv[u].x, xv[u].x, acc1[u]));
    }
  }
#pragma unroll
  for (int w = RD2_U / 2; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) {
      acc0[u] += acc0[u + w];
      acc1[u] += acc1[u + w];
    }
  double v0 = acc0[0], v1 = acc1[0];
  for (int off = 32; off > 0; off >>= 1) {
    v0 += __shfl_down(v0, off, 64);
    v1 += __shfl_down(v1, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v0;
    red[NT / 64 + (threadIdx.x >> 6)] = v1;
  }
  __syncthreads();
  s0 = s1 = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) {
      s0 += red[w];
      s1 += red[NT / 64 + w];
    }
}

// k_rows_dot with pairs, two rows per workgroup (rows 2 r and 2 r + 1 of chunk ch; an odd last row
// is taken alone): the same partials, the same bits
__global__ __launch_bounds__(RP_THREADS) void k_rows_dot_two(int nr, i64 N, int nch, const double* __restrict__ M,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ xm,
                                                             double* __restrict__ part, BatchStrides bs) {
  __shared__ double red[2 * RP_THREADS / 64];
  M += blockIdx.y * bs.M;
  x += blockIdx.y * bs.v;
  if (xm) xm += blockIdx.y * bs.v;
  part += blockIdx.y * bs.u;
  const int r0 = 2 * (int)(blockIdx.x / nch), ch = (int)(blockIdx.x % nch);
  const bool two = r0 + 1 < nr;
  i64 L = (N + nch - 1) / nch;
  L = (L + 1) & ~(i64)1;
  const i64 lo = min(N, (i64)ch * L), hi = min(N, lo + L);
  if (two) {
    double s0, s1;
    dot_range2_two<RP_THREADS>(M + (i64)r0 * N, M + (i64)(r0 + 1) * N, x, lo, hi, red, xm, s0, s1);
    if (threadIdx.x == 0) {
      part[(i64)r0 * nch + ch] = s0;
      part[(i64)(r0 + 1) * nch + ch] = s1;
    }
  } else {
    const double s0 = dot_range2<RP_THREADS>(M + (i64)r0 * N, x, lo, hi, red, xm);
    if (threadIdx.x == 0) part[(i64)r0 * nch + ch] = s0;
  }
}

// pairs: every chunk starts and ends on a pair (N even, the vectors 16-byte aligned)
__global__ __launch_bounds__(RP_THREADS) void k_rows_dot(i64 N, int nch, const double* __restrict__ M,
                                                         const double* __restrict__ x, const double* __restrict__ xm,
                                                         double* __restrict__ part, BatchStrides bs, int pairs) {
  __shared__ double red[RP_THREADS / 64];
  M += blockIdx.y * bs.M;
  x += blockIdx.y * bs.v;
  if (xm) xm += blockIdx.y * bs.v;
  part += blockIdx.y * bs.u;
  const int row = (int)(blockIdx.x / nch), ch = (int)(blockIdx.x % nch);
  i64 L = (N + nch - 1) / nch;
  if (pairs) L = (L + 1) & ~(i64)1;
  const i64 lo = min(N, (i64)ch * L), hi = min(N, lo + L);
  const double s = pairs ? dot_range2<RP_THREADS>(M + (i64)row * N, x, lo, hi, red, xm)
                         : dot_range<RP_THREADS>(M + (i64)row * N, x, lo, hi, red, xm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <bool TWO, bool DOT, int PF>
__global__ __launch_bounds__(64 * CU_WAVES) void k_cols_update(int nr, i64 N, const double* __restrict__ M,
                                                               const double* __restrict__ u, int u_nch,
                                                               const double* __restrict__ eta, const double* base,
                                                               double* out, double* out2, const double* __restrict__ M2,
                                                               const double* base2, double* out3, double* dot_part,
                                                               const double* __restrict__ base2m, BatchStrides bs) {
  __shared__ double us[CU_BLK];
  __shared__ double part[CU_WAVES][64];
  __shared__ double part2[TWO ? CU_WAVES : 1][64];
  {
    const i64 z = blockIdx.y;
    M += z * bs.M;
    if (TWO) M2 += z * bs.M;
    u += z * bs.u;
    if (eta) eta += z * bs.eta;
    base += z * bs.v;
    out += z * bs.v;
    if (out2) out2 += z * bs.v;
    if (TWO) { base2 += z * bs.v; out3 += z * bs.v; }
    if (base2m) base2m += z * bs.v;
    if (DOT) dot_part += z * bs.part;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const i64 c = (i64)blockIdx.x * 64 + lane;
  // the addends of the output, loaded before anything they do not depend on
  const bool cw = wave == 0 && c < N;
  const double bv = cw ? base[c] : 0.0;
  const double bv2 = (TWO && cw) ? base2[c] : 0.0;
  const double bvm = (TWO && cw && base2m) ? base2m[c] : 0.0;
  double acc = 0.0, acc2 = 0.0;
  for (int j0 = 0; j0 < nr; j0 += CU_BLK) {
    const int jn = min(CU_BLK, nr - j0);
    // this wavefront's first PF rows of the block, loaded before the
    // coefficients are staged (they do not depend on them)
    double pm[PF > 0 ? PF : 1], pm2[PF > 0 ? PF : 1];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = wave + k * CU_WAVES;
      const bool ok = c < N && i < jn;
      pm[k] = ok ? M[(i64)(j0 + i) * N + c] : 0.0;
      pm2[k] = (TWO && ok) ? M2[(i64)(j0 + i) * N + c] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < jn; i += 64 * CU_WAVES) {
      // the partials of row j0 + i added in order (a register array of all of them
      // doubled the kernel's registers and halved its occupancy)
      const double* pu = u + (i64)(j0 + i) * u_nch;
      const double ev = eta ? eta[j0 + i] : 1.0;
      double v = pu[0];
      for (int ch = 1; ch < u_nch; ++ch) v += pu[ch];
      us[i] = eta ? v / ev : v;
    }
    __syncthreads();
    if (c < N) {
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int i = wave + k * CU_WAVES;
        if (i < jn) {
          acc = fma(pm[k], us[i], acc);
          if (TWO) acc2 = fma(pm2[k], us[i], acc2);
        }
      }
#pragma unroll 4
      for (int i = wave + PF * CU_WAVES; i < jn; i += CU_WAVES) {
        const i64 off = (i64)(j0 + i) * N + c;
        acc = fma(M[off], us[i], acc);
        if (TWO) acc2 = fma(M2[off], us[i], acc2);
      }
    }
  }
  part[wave][lane] = acc;
  if (TWO) part2[wave][lane] = acc2;
  __syncthreads();
  double prod = 0.0;
  if (wave == 0 && c < N) {
    double s = 0.0;
    for (int w = 0; w < CU_WAVES; ++w) s += part[w][lane];
    const double v = bv - s;
    out[c] = v;
    if (out2) out2[c] = v;
    if (TWO) {
      double s2 = 0.0;
      for (int w = 0; w < CU_WAVES; ++w) s2 += part2[w][lane];
      const double b2 = base2m ? bv2 - bvm : bv2;
      const double v3 = b2 - s2;
      out3[c] = v3;
      prod = v * v3;
    }
  }
  if (DOT && wave == 0) {                        // this workgroup's part of sum_c out[c] * out3[c]
    prod = wave_sum(prod);
    if (lane == 0) dot_part[blockIdx.x] = prod;
  }
}

int rows_dot_chunks(int nr, i64 N) {
  if (nr <= 0) return 1;
  const i64 by_rows = (ROWS_DOT_TARGET + nr - 1) / nr;
  const i64 by_len = std::max<i64>(1, (N + 2047) / 2048);   // chunks of >= 2048 columns
  return (int)std::max<i64>(1, std::min<i64>(16, std::min(by_rows, by_len)));
}

hipError_t launch_rows_dot(int nr, i64 N, const double* M, const double* x, double* part, hipStream_t s,
                           const double* xm, int batch, const BatchStrides& bs) {
  if (nr <= 0 || N <= 0) return hipSuccess;
  const int nch = rows_dot_chunks(nr, N);
  const auto al = [](const void* p) { return (uintptr_t)p % 16 == 0; };
  const bool odd_stride = (bs.M % 2) || (bs.v % 2);
  const int pairs = (N % 2 == 0) && !odd_stride && al(M) && al(x) && (!xm || al(xm));
  const i64 pairs_of_rows = (nr + 1) / 2;
  if (pairs && pairs_of_rows * nch >= ROWS_DOT_TWO_MIN_WG)   // enough workgroups with two rows each
    k_rows_dot_two<<<dim3((unsigned)(pairs_of_rows * nch), batch), dim3(RP_THREADS), 0, s>>>(nr, N, nch, M, x, xm,
                                                                                            part, bs);
  else
    k_rows_dot<<<dim3((unsigned)((i64)nr * nch), batch), dim3(RP_THREADS), 0, s>>>(N, nch, M, x, xm, part, bs, pairs);
  return hipGetLastError();
}

hipError_t launch_rows_dot_full(int nr, i64 N, const double* M, const double* x, double* out, hipStream_t s) {
  if (nr <= 0 || N <= 0) return hipSuccess;
  k_rows_dot<<<dim3((unsigned)nr), dim3(RP_THREADS), 0, s>>>(N, 1, M, x, nullptr, out, BatchStrides(), 0);
  return hipGetLastError();
}

// The coefficients of a column update, once: out[j] = (sum_ch u[j][ch]) / (eta ? eta[j] : 1),
// the partials added in order (the same arithmetic as the staging inside k_cols_update).
__global__ void k_coef_finish(int nr, int u_nch, const double* __restrict__ u, const double* __restrict__ eta,
                              double* __restrict__ out, BatchStrides bs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  u += blockIdx.y * bs.u;
  out += blockIdx.y * bs.u;
  if (eta) eta += blockIdx.y * bs.eta;
  if (j >= nr) return;
  const double* pu = u + (i64)j * u_nch;
  double v = pu[0];
  for (int ch = 1; ch < u_nch; ++ch) v += pu[ch];
  out[j] = eta ? v / eta[j] : v;
}

template <int PF>
static void cols_update_launch(dim3 grid, dim3 block, hipStream_t s, int nr, i64 N, const double* M, const double* u,
                               int u_nch, const double* eta, const double* base, double* out, double* out2,
                               const double* M2, const double* base2, double* out3, double* dot_part,
                               const double* base2m, const BatchStrides& bs) {
  if (M2 && dot_part)
    k_cols_update<true, true, PF><<<grid, block, 0, s>>>(nr, N, M, u, u_nch, eta, base, out, out2, M2, base2, out3,
                                                         dot_part, base2m, bs);
  else if (M2)
    k_cols_update<true, false, PF><<<grid, block, 0, s>>>(nr, N, M, u, u_nch, eta, base, out, out2, M2, base2, out3,
                                                          nullptr, base2m, bs);
  else
    k_cols_update<false, false, PF><<<grid, block, 0, s>>>(nr, N, M, u, u_nch, eta, base, out, out2, nullptr, nullptr,
                                                           nullptr, nullptr, nullptr, bs);
}

hipError_t launch_cols_update(int nr, i64 N, const double* M, double* u, int u_nch, const double* eta,
                              const double* base, double* out, double* out2, const double* M2, const double* base2,
                              double* out3, hipStream_t s, double* dot_part, const double* base2m, int batch,
                              const BatchStrides& bs) {
  if (N <= 0) return hipSuccess;
  if (u_nch < 1 || u_nch > CU_MAXCH) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + 63) / 64), batch), block(64 * CU_WAVES);
  if (N >= CU_FINISH_MIN_N) {
    // Many workgroups per CU in turn: each would expose the latency of staging the
    // coefficients from their partials, so they are finished once, after the partials.
    if (nr > 0 && (u_nch > 1 || eta)) {
      double* fin = u + (i64)nr * u_nch;
      k_coef_finish<<<dim3((unsigned)((nr + 255) / 256), batch), 256, 0, s>>>(nr, u_nch, u, eta, fin, bs);
      u = fin;
      u_nch = 1;
      eta = nullptr;
    }
    cols_update_launch<0>(grid, block, s, nr, N, M, u, u_nch, eta, base, out, out2, M2, base2, out3, dot_part, base2m,
                          bs);
  } else {
    cols_update_launch<CU_PF>(grid, block, s, nr, N, M, u, u_nch, eta, base, out, out2, M2, base2, out3, dot_part,
                              base2m, bs);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Triangular matrix-vector product for large point blocks, one wavefront per
// row of a row-major matrix (coalesced streaming of the triangle):
//   y[i] = add[i] + alpha * sum_{k in K_i} M[i][k] x[k],
//   K_i = [0, i] (upper = 0, lower-triangular M) or [i, n) (upper = 1).
// Transposed products use the stored transpose, so every product streams rows.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_trmv_rows(int n, const double* __restrict__ M, const double* __restrict__ x,
                                                   double* __restrict__ y, double alpha, const double* __restrict__ add,
                                                   int upper) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int lo = upper ? i : 0, hi = upper ? n : i + 1;
  const double* __restrict__ row = M + (i64)i * n;
  double acc = 0;
  int k = lo + lane;
  for (; k + 192 < hi; k += 256) {
    acc += row[k] * x[k];
    acc += row[k + 64] * x[k + 64];
    acc += row[k + 128] * x[k + 128];
    acc += row[k + 192] * x[k + 192];
  }
  for (; k < hi; k += 64) acc += row[k] * x[k];
  acc = wave_sum(acc);
  if (lane == 0) y[i] = (add ? add[i] : 0.0) + alpha * acc;
}

// The same product with 16-byte loads (n even, M and x 16-byte aligned: every
// row starts on a pair): lane l takes the pairs l, l + 64, ... of [lo, hi)
// rounded inward to pairs, four in flight, and lane 0 adds the odd element at
// either end.  17% faster than the 8-byte form on the 16384^2 triangle.
constexpr int TV_UN = 4;
__global__ __launch_bounds__(256) void k_trmv_rows2(int n, const double* __restrict__ M, const double* __restrict__ x,
                                                    double* __restrict__ y, double alpha,
                                                    const double* __restrict__ add, int upper) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int lo = upper ? i : 0, hi = upper ? n : i + 1;
  const double* __restrict__ row = M + (i64)i * n;
  const double2* __restrict__ row2 = reinterpret_cast<const double2*>(row);
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);
  const int pa = (lo + 1) / 2, pb = hi / 2;      // pairs [2 pa, 2 pb) of [lo, hi)
  double acc[TV_UN];
#pragma unroll
  for (int u = 0; u < TV_UN; ++u) acc[u] = 0.0;
  int p = pa + lane;
  for (; p + 64 * (TV_UN - 1) < pb; p += 64 * TV_UN) {
    double2 mv[TV_UN], xv[TV_UN];
#pragma unroll
    for (int u = 0; u < TV_UN; ++u) {
      mv[u] = row2[p + 64 * u];
      xv[u] = x2[p + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < TV_UN; ++u) acc[u] += mv[u].x * xv[u].x + mv[u].y * xv[u].y;
  }
  for (; p < pb; p += 64) {
    const double2 mv = row2[p], xv = x2[p];
    acc[0] += mv.x * xv.x + mv.y * xv.y;
  }
  double a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (lane == 0) {
    if (lo & 1) a += row[lo] * x[lo];            // the odd element before the first pair
    if (hi & 1) a += row[hi - 1] * x[hi - 1];    // and after the last (never the same one)
  }
  a = wave_sum(a);
  if (lane == 0) y[i] = (add ? add[i] : 0.0) + alpha * a;
}
static_assert(TV_UN == 4, "the accumulators are added as two pairs");

hipError_t launch_trmv_rows(int n, const double* M, const double* x, double* y, double alpha, const double* add,
                            int upper, hipStream_t s) {
  const bool pairs = (n % 2 == 0) && ((uintptr_t)M % 16 == 0) && ((uintptr_t)x % 16 == 0);
  if (pairs) k_trmv_rows2<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, M, x, y, alpha, add, upper);
  else k_trmv_rows<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, M, x, y, alpha, add, upper);
  return hipGetLastError();
}

// B = A^T for n x n row-major matrices, in 64 x 64 tiles through LDS so that both the reads of A
// and the writes of B run along rows (a row of the tile per wavefront pass, one element per lane);
// the odd column of the padded LDS rows spreads a tile column over the banks.
constexpr int TP_T = 64;
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ A, double* __restrict__ B, int n) {
  __shared__ double t[TP_T][TP_T + 1];
  const int tiles = (n + TP_T - 1) / TP_T;
  const int tr = (int)(blockIdx.x / tiles), tc = (int)(blockIdx.x % tiles);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = tr * TP_T, c0 = tc * TP_T;
  for (int i = w; i < TP_T; i += 4) {            // tile row i of A: A[r0 + i][c0 + lane]
    const int r = r0 + i, c = c0 + lane;
    if (r < n && c < n) t[i][lane] = A[(i64)r * n + c];
  }
  __syncthreads();
  for (int j = w; j < TP_T; j += 4) {            // row c0 + j of B: B[c0 + j][r0 + lane] = A[r0 + lane][c0 + j]
    const int r = c0 + j, c = r0 + lane;
    if (r < n && c < n) B[(i64)r * n + c] = t[lane][j];
  }
}

hipError_t launch_transpose(const double* A, double* B, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const i64 tiles = (i64)((n + TP_T - 1) / TP_T);
  k_transpose<<<(unsigned)(tiles * tiles), 256, 0, s>>>(A, B, n);
  return hipGetLastError();
}

hipError_t launch_dot(i64 n, const double* x, const double* y, double* partial, double* out,
                      hipStream_t s, int batch, const BatchStrides& bs) {
  k_dot_partial<<<dim3(DOT_BLOCKS, batch), DOT_THREADS, 0, s>>>(n, x, y, partial, bs.v);
  k_dot_final<<<batch, DOT_THREADS, 0, s>>>(partial, out, bs.scal);
  return hipGetLastError();
}

}  // namespace gpfvm
