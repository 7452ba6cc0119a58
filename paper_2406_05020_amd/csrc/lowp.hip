// Grouped GEMM of the low-precision volume operator on the bfloat16 matrix
// cores (descriptor semantics in common.h; float32 operands in HBM).
//
// The Gram factors and the tensor they multiply are float32.  On the way into
// LDS every float32 value a is split into three bfloat16 slices,
//   a = s1 + s2 + s3 + O(2^-24 |a|),  s1 = bf16(a), s2 = bf16(a - s1),
//   s3 = bf16(a - s1 - s2)
// (round to nearest even; each remainder is exact in float32), and a 16x16
// output block takes the six slice products whose orders sum to at most 4,
//   A1 B1 + (A1 B2 + A2 B1 + A1 B3 + A2 B2 + A3 B1),
// on v_mfma_f32_16x16x32_bf16 with float32 accumulation.  A bfloat16 product
// is exact in float32, so the result carries float32 accuracy: the dropped
// products are below 2^-24 of |A||B|.  A single bfloat16 slice (2^-9) would
// leave the volume system indefinite: the Gram's small eigenvalues sit at the
// noise level, about 1e-6 of its mean diagonal.
//
// Lane layout of the 16x16x32 bfloat16 MFMA on gfx950 (checked by a lane
// probe): lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16],
// j < 8; accumulator register r of lane l holds D[4 (l / 16) + r][l % 16].
#include <hip/hip_runtime.h>

#include "common.h"

namespace gpfvm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int BS_KC = 32;            // K per chunk: one MFMA step
constexpr int BS_LD = BS_KC + 8;     // LDS row stride (bf16 elements): 80 bytes, 16-byte aligned rows
constexpr int BS_THREADS = 256;      // four wavefronts

// bfloat16 bits of x rounded to nearest even (x finite)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ void split3(float a, unsigned short& s1, unsigned short& s2, unsigned short& s3) {
  s1 = bf16_bits(a);
  const float r1 = a - bf16_value(s1);
  s2 = bf16_bits(r1);
  const float r2 = r1 - bf16_value(s2);
  s3 = bf16_bits(r2);
}

__device__ __forceinline__ bf16x8 frag(const unsigned short* p) {
  const u16x8 v = *reinterpret_cast<const u16x8*>(p);
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Tiles dealt to the XCDs in chunks of four (the same bijection as the float64 GEMM).
__device__ __forceinline__ i64 bs_xcd_tile(i64 w, i64 n) {
  const i64 full = n / 32 * 32;
  if (w >= full) return w;
  const i64 x = w % 8, j = w / 8;
  return ((j / 4) * 8 + x) * 4 + j % 4;
}

// BM x BM output tile per workgroup; the four wavefronts form a 2 x 2 grid of
// (BM/2) x (BM/2) sub-tiles, each WB x WB blocks of 16 x 16.
template <int BM>
__global__ __launch_bounds__(BS_THREADS) void k_gemm_bf16s(const GemmDesc* __restrict__ descs, int ndesc,
                                                           i64 ntiles) {
  constexpr int WB = BM / 32;                        // 16x16 blocks per wavefront and direction
  constexpr int EA = BM * BS_KC / BS_THREADS;        // float32 elements of A (and of B) per thread
  // 16-byte aligned: every lane reads its eight k of a row as one 16-byte load
  __shared__ __attribute__((aligned(16))) unsigned short As[3][BM][BS_LD];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[3][BM][BS_LD];

  const i64 tile = bs_xcd_tile(blockIdx.x, ntiles);
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
  const int M = D.M, N = D.N;
  const int m0 = tm * BM, n0 = tn * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * (BM / 2);

  // [slot][block row][block col]: leading product and the five correction products
  f32x4 acc[2][WB][WB], acl[2][WB][WB];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
      for (int j = 0; j < WB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][i][j][r] = acl[q][i][j][r] = 0.0f;
  bool used1 = false;

  for (int g = 0; g < D.nseg; ++g) {
    const Seg& S = D.seg[g];
    const float* __restrict__ A = reinterpret_cast<const float*>(S.A) + b * S.a_bs;
    const float* __restrict__ B = reinterpret_cast<const float*>(S.B) + b * S.b_bs;
    const i64 a_rs = S.a_rs, a_cs = S.a_cs, b_rs = S.b_rs, b_cs = S.b_cs;
    const float alpha = (float)S.alpha;
    const int q = S.slot ? 1 : 0;
    used1 |= (q == 1);
    int kbeg = 0, kend = S.K;
    if (S.tri == 1) kend = min(S.K, m0 + BM);
    else if (S.tri == 2) kbeg = m0;
    else if (S.tri == 3) kend = min(S.K, n0 + BM);
    else if (S.tri == 4) kbeg = n0;
    if (kbeg >= kend) continue;
    const bool akf = (a_cs == 1), bnf = (b_cs == 1);
    float ra[EA], rb[EA];
    // chunk kc of both operands into registers (zero outside the tile and the K range)
    auto gload = [&](int kc) {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + BS_THREADS * u;
        int k, m;
        if (akf) { k = e % BS_KC; m = e / BS_KC; } else { m = e % BM; k = e / BM; }
        ra[u] = (m0 + m < M && kc + k < kend) ? alpha * A[(i64)(m0 + m) * a_rs + (i64)(kc + k) * a_cs] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + BS_THREADS * u;
        int k, n;
        if (bnf) { n = e % BM; k = e / BM; } else { k = e % BS_KC; n = e / BS_KC; }
        rb[u] = (n0 + n < N && kc + k < kend) ? B[(i64)(kc + k) * b_rs + (i64)(n0 + n) * b_cs] : 0.0f;
      }
    };
    auto sstore = [&]() {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + BS_THREADS * u;
        int k, m;
        if (akf) { k = e % BS_KC; m = e / BS_KC; } else { m = e % BM; k = e / BM; }
        split3(ra[u], As[0][m][k], As[1][m][k], As[2][m][k]);
      }
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + BS_THREADS * u;
        int k, n;
        if (bnf) { n = e % BM; k = e / BM; } else { k = e % BS_KC; n = e / BS_KC; }
        split3(rb[u], Bs[0][n][k], Bs[1][n][k], Bs[2][n][k]);
      }
    };
    __syncthreads();                   // the previous segment's last chunk has been read
    gload(kbeg);
    for (int kc = kbeg; kc < kend; kc += BS_KC) {
      sstore();
      __syncthreads();
      if (kc + BS_KC < kend) gload(kc + BS_KC);     // next chunk in flight during the products
#pragma unroll
      for (int i = 0; i < WB; ++i) {
        const int row = wr + 16 * i + lr;
        const bf16x8 a1 = frag(&As[0][row][8 * lk]), a2 = frag(&As[1][row][8 * lk]), a3 = frag(&As[2][row][8 * lk]);
#pragma unroll
        for (int j = 0; j < WB; ++j) {
          const int col = wc + 16 * j + lr;
          const bf16x8 b1 = frag(&Bs[0][col][8 * lk]), b2 = frag(&Bs[1][col][8 * lk]),
                       b3 = frag(&Bs[2][col][8 * lk]);
          f32x4 h = acc[q][i][j], c = acl[q][i][j];
          h = mfma(a1, b1, h);
          c = mfma(a1, b2, c);
          c = mfma(a2, b1, c);
          c = mfma(a1, b3, c);
          c = mfma(a2, b2, c);
          c = mfma(a3, b1, c);
          acc[q][i][j] = h;
          acl[q][i][j] = c;
        }
      }
      __syncthreads();                 // every wavefront is done with this chunk
    }
  }

  float* __restrict__ C = reinterpret_cast<float*>(D.C) + b * D.c_bs;
  const float* __restrict__ X = D.X ? reinterpret_cast<const float*>(D.X) + b * D.x_bs : nullptr;
  const double* __restrict__ E = D.escale ? D.escale + b * D.e_bs : nullptr;
  const float beta = (float)D.beta, gamma = (float)D.gamma;
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * i + 4 * lk + r;
        const int col = n0 + wc + 16 * j + lr;
        if (row < M && col < N && !(D.lower_only && col > row)) {
          float v = acc[0][i][j][r] + acl[0][i][j][r];
          if (used1 && E) v += (float)E[(i64)row * D.e_rs + (i64)col * D.e_cs] * (acc[1][i][j][r] + acl[1][i][j][r]);
          if (X) v += gamma * X[(i64)row * D.x_rs + (i64)col * D.x_cs];
          float* cp = C + (i64)row * D.c_rs + (i64)col * D.c_cs;
          if (beta != 0.0f) v += beta * *cp;
          *cp = v;
        }
      }
}

}  // namespace

hipError_t launch_gemm_bf16s(const Stage& st, hipStream_t s) {
  if (st.tiles == 0 || st.descs.empty()) return hipSuccess;
  if (st.rider.kind != RIDE_NONE) return hipErrorInvalidValue;     // float64 riders only
  const int nd = (int)st.descs.size();
  const dim3 grid((unsigned)st.tiles), block(BS_THREADS);
  if (st.kind == GEMM_BF16S64) k_gemm_bf16s<64><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles);
  else k_gemm_bf16s<32><<<grid, block, 0, s>>>(st.d_descs, nd, st.tiles);
  return hipGetLastError();
}

}  // namespace gpfvm
