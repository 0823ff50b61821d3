// Normal matrix M = A D A^T of the Section 5 normal equations on the FP64
// matrix cores of gfx950, and the same tile routine (syrk_tile.h) in
// subtract mode for the Cholesky trailing update.
//
// Two FP64 families:
//   * k_syrk_sk (below): stream-K over 128 x 128 lower tiles on
//     v_mfma_f64_16x16x4f64, the choice for large shapes;
//   * k_syrk_f64: split-K over 64 or 128 lower tiles with the four-block
//     v_mfma_f64_4x4x4f64 tile routine of syrk_tile.h (small shapes and the
//     Cholesky updates);
//   * k_bsyrk_normal16 / k_bsyrk_normal_sk: the batched normal matrices,
//     one LP per workgroup row of tiles, on the 16x16x4 form.
// Split-K writes per-split partial tiles; the last split of a tile to finish
// (an arrival counter per tile) sums them in split order, so results do not
// depend on scheduling.  The FP32 kernel (mixed precision) is further down.
#include <algorithm>
#include <cmath>

#include "pdas_internal.h"
#include "syrk_tile.h"

namespace pdas {
namespace {

template <int R, int Q, int KC, bool SCALE, bool VEC>
__global__ __launch_bounds__(256) void k_syrk_f64(int mm, int K, const double* __restrict__ X,
                                                  long ldx, const double* __restrict__ w,
                                                  double* __restrict__ C, long ldc, int sub,
                                                  int ntiles, int per_xcd, int kchunk,
                                                  double* __restrict__ part) {
  // XCD-aware order: consecutive tiles (sharing row panels) on one XCD.
  __shared__ double2 lds2[syrk_tile_lds2<R, KC>()];
  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= ntiles) return;
  syrk_f64_tile<R, Q, KC, SCALE, VEC>(mm, K, X, ldx, w, C, ldc, sub, t, ntiles, blockIdx.y,
                                      gridDim.y, kchunk, part, lds2);
}

// ---------------------------------------------------------------------------
// FP32 normal matrix (mixed precision): M32 = (A32 diag(sd)) (A32 diag(sd))^T
// with sd = sqrt(d) applied to both operands while staging (column scaling by
// the square root of D keeps the FP32 operands balanced), and the same kernel
// in subtract mode for the FP32 Cholesky trailing update.
//
// Instruction: v_mfma_f32_16x16x4f32.  Lane l holds
//   A operand: rowop[i = l % 16][k = l / 16],
//   B operand: colop[j = l % 16][k = l / 16],
//   D result : 4 values, C[i = 4 (l / 16) + v][j = l % 16].
// A wavefront owns a (16 R) x (16 R) output (R x R blocks); a workgroup of
// 2 x 2 wavefronts owns a BM = 32 R square tile.  LDS layout as in the FP64
// kernel (blocks of 4 k by 16 rows), so every operand read is lane-linear.
// One lower tile t (linear index over the lower triangle of BM-tiles) and
// K split `split` of the FP32 product; the whole workgroup takes part.
// lds: the caller's [2 stages][2 operands][BM * KC] floats.
template <int R, int KC, bool SCALE>
__device__ __forceinline__ void syrk_f32_tile(int mm, int K, const float* __restrict__ X,
                                              long ldx, const float* __restrict__ w,
                                              float* __restrict__ C, long ldc, int sub, int t,
                                              int split, int ntiles, int kchunk,
                                              float* __restrict__ part,
                                              float (*lds)[2][32 * R * KC]) {
  constexpr int BM = 32 * R;
  constexpr int QPR = KC / 4;              // float4 groups per row per stage
  constexpr int QUADS = BM * QPR / 256;    // groups per thread per operand
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nst = (kend - kbeg + KC - 1) / KC;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv >> 1) * (16 * R), wc0 = (wv & 1) * (16 * R);
  const bool active = !(ti == tj && wr0 + 16 * R <= wc0);

  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 acc[R][R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};

  float4 pa[QUADS], pb[QUADS], pw[QUADS];
  // Requires K % 4 == 0 and 16-byte aligned rows (checked by the launcher).
  auto gload = [&](int st) {
    const int kb = kbeg + st * KC;
#pragma unroll
    for (int it = 0; it < QUADS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / QPR, k = kb + 4 * (p % QPR);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      const int kc = min(k, kend - 4);
      pa[it] = *reinterpret_cast<const float4*>(X + ra * ldx + kc);
      pb[it] = *reinterpret_cast<const float4*>(X + rb * ldx + kc);
      if (SCALE) pw[it] = *reinterpret_cast<const float4*>(w + kc);
    }
  };
  auto sstore = [&](int buf, int st) {
    const int kb = kbeg + st * KC;
#pragma unroll
    for (int it = 0; it < QUADS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / QPR, kk = 4 * (p % QPR), k = kb + kk;
      const bool va = row0 + row < mm && k < kend, vb = col0 + row < mm && k < kend;
      float a[4] = {pa[it].x, pa[it].y, pa[it].z, pa[it].w};
      float bb[4] = {pb[it].x, pb[it].y, pb[it].z, pb[it].w};
      if (SCALE) {
        const float ww[4] = {pw[it].x, pw[it].y, pw[it].z, pw[it].w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          a[v] *= ww[v];
          bb[v] *= ww[v];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        lds[buf][0][lidx<BM>(row, kk + v)] = va ? a[v] : 0.f;
        lds[buf][1][lidx<BM>(row, kk + v)] = vb ? bb[v] : 0.f;
      }
    }
  };

  if (nst > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload(st + 1);
    if (active) {
      const float* la = lds[cur][0];
      const float* lb = lds[cur][1];
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        float bq[R];
#pragma unroll
        for (int c = 0; c < R; ++c) bq[c] = lb[lidx<BM>(wc0 + 16 * c + li, 4 * ks + lk)];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float av = la[lidx<BM>(wr0 + 16 * r + li, 4 * ks + lk)];
#pragma unroll
          for (int c = 0; c < R; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[c], acc[r][c], 0, 0, 0);
        }
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1, st + 1);
    __syncthreads();
  }

  if (!active) return;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wr0 + 16 * r + 4 * lk + v, lc = wc0 + 16 * c + li;
        if (part) {
          part[((long)split * ntiles + t) * (BM * BM) + lr * BM + lc] = acc[r][c][v];
        } else {
          const int gr = row0 + lr, gc = col0 + lc;
          if (gr < mm && gc <= gr) {
            float* cp = C + (long)gr * ldc + gc;
            *cp = sub ? (*cp - acc[r][c][v]) : acc[r][c][v];
          }
        }
      }
}

template <int R, int KC, bool SCALE>
__global__ __launch_bounds__(256) void k_syrk_f32(int mm, int K, const float* __restrict__ X,
                                                  long ldx, const float* __restrict__ w,
                                                  float* __restrict__ C, long ldc, int sub,
                                                  int ntiles, int per_xcd, int kchunk,
                                                  float* __restrict__ part) {
  __shared__ float lds[2][2][32 * R * KC];
  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= ntiles) return;
  syrk_f32_tile<R, KC, SCALE>(mm, K, X, ldx, w, C, ldc, sub, t, blockIdx.y, ntiles, kchunk, part,
                              lds);
}

template <int BM>
__global__ __launch_bounds__(256) void k_syrk_reduce_f32(int mm, float* __restrict__ C, long ldc,
                                                         int sub, int ntiles, int splits,
                                                         const float* __restrict__ part) {
  const int t = blockIdx.x;
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  for (int e = threadIdx.x; e < BM * BM; e += 256) {
    const int lr = e / BM, lc = e % BM;
    const int gr = row0 + lr, gc = col0 + lc;
    if (gr >= mm || gc > gr) continue;
    float v = 0.f;
    for (int s = 0; s < splits; ++s) v += part[((long)s * ntiles + t) * (BM * BM) + e];
    float* cp = C + (long)gr * ldc + gc;
    *cp = sub ? (*cp - v) : v;
  }
}

constexpr int kKC128 = 32;  // K per stage of the 128 x 128 tile kernel
constexpr int kKC64 = 32;   // and of the 64 x 64 one

// Batched Cholesky trailing update after the panel at column p:
// M22 -= L21 L21^T on the lower BM-tiles of each LP that has rows below p + 64.
template <int BM>
__global__ __launch_bounds__(256) void k_bsyrk_trailing(const BatchLP* __restrict__ lps,
                                                         const int* __restrict__ go,
                                                         double* __restrict__ Mpool, int p) {
  const int lp = blockIdx.y;
  if (!go[lp]) return;
  const BatchLP P = lps[lp];
  const int mm = P.m - p - 64;
  if (mm <= 0) return;
  const int nt = (mm + BM - 1) / BM, ntiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  double* X = Mpool + P.M_off + (long)(p + 64) * P.ldm + p;
  __shared__ double2 lds2[syrk_tile_lds2<BM / 8, 32>()];
  syrk_f64_tile<BM / 8, BM / 32, 32, false, true>(mm, 64, X, P.ldm, nullptr, X + 64, P.ldm, 1, t,
                                                  ntiles, 0, 1, 64, nullptr, lds2);
}

// Batched FP32 normal matrices (mixed precision): LP = blockIdx.y, lower
// BM-tile blockIdx.x of M32_i = (A32_i diag(sd_i)) (A32_i diag(sd_i))^T over
// the padded rows (n4 = n rounded up to 4, zero padding), for the LPs whose
// flag is set.
template <int R>
__global__ __launch_bounds__(256) void k_bsyrk_normal_f32(const BatchLP* __restrict__ lps,
                                                           const int* __restrict__ go,
                                                           const float* __restrict__ A32,
                                                           const float* __restrict__ sd32,
                                                           float* __restrict__ M32) {
  const int lp = blockIdx.y;
  if (!go[lp]) return;
  const BatchLP P = lps[lp];
  constexpr int BM = 32 * R;
  const int nt = (P.m + BM - 1) / BM, ntiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  __shared__ float lds[2][2][32 * R * 32];
  syrk_f32_tile<R, 32, true>(P.m, P.n4, A32 + P.a32_off, P.n4, sd32 + P.vn4, M32 + P.m32_off,
                             P.ld32, 0, t, 0, ntiles, P.n4, nullptr, lds);
}

// Batched FP32 trailing update after the panel at column p.
template <int R>
__global__ __launch_bounds__(256) void k_bsyrk_trailing_f32(const BatchLP* __restrict__ lps,
                                                             const int* __restrict__ go,
                                                             float* __restrict__ M32, int p) {
  const int lp = blockIdx.y;
  if (!go[lp]) return;
  const BatchLP P = lps[lp];
  const int mm = P.m - p - 64;
  if (mm <= 0) return;
  constexpr int BM = 32 * R;
  const int nt = (mm + BM - 1) / BM, ntiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  float* X = M32 + P.m32_off + (long)(p + 64) * P.ld32 + p;
  __shared__ float lds[2][2][32 * R * 32];
  syrk_f32_tile<R, 32, false>(mm, 64, X, P.ld32, nullptr, X + 64, P.ld32, 1, t, 0, ntiles, 64,
                              nullptr, lds);
}

// ---------------------------------------------------------------------------
// Stream-K normal matrix on v_mfma_f64_16x16x4f64 (lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; slot v of the result is
// D[l / 16 + 4 v][l % 16]).  The 16x16 product has no replicated operand, so
// a K-step of a wavefront's 64 x 32 block needs 6 LDS reads for 8
// instructions (the 4x4x4 form needs 18 for the same work); that is what
// keeps this kernel off the LDS bandwidth limit.
//
// Workgroup tile 128 x 128 (2 x 4 wavefronts of 64 x 32), stages of 32 along
// K through double-buffered LDS rows padded to 33 doubles.  The iteration
// space (lower tiles x stages, tile-major) is cut into kSkGroups equal
// contiguous ranges, one per workgroup, so every compute unit gets the same
// amount of matrix work whatever the number of tiles.  A range covers the
// end of one tile, whole tiles and the start of another: whole tiles are
// written directly; a partial tile goes to the workgroup's slot (first or
// last) and the last of the tile's workgroups to arrive (a counter per tile)
// adds the slots in workgroup order, so the result does not depend on
// scheduling; that workgroup adds the other slots to its own segment, still
// in registers, with lane-contiguous loads.  Consecutive workgroup ids land
// on different XCDs; the range index is remapped so that each XCD owns one
// contiguous eighth of the work.
constexpr int kSkT = 4;                 // 16 x 16 blocks per wavefront, rows
constexpr int kSkBM = 32 * kSkT;        // 128
constexpr int kSkKC = 32;
constexpr int kSkLS = kSkKC + 1;     // odd: the 16 rows of an operand read fall in distinct banks
constexpr int kSkGroups = 256;          // one workgroup per compute unit

typedef double sk4 __attribute__((ext_vector_type(4)));

// Wavefront grid of a workgroup: 2 x WC wavefronts, each a 64 x (128 / WC)
// part of the tile (kSkT x TC blocks of 16 x 16).  With WC = 4 (eight
// wavefronts, 222 registers each) two wavefronts share each SIMD, so one
// wavefront's operand reads and barrier waits overlap the other's matrix
// work; measured 9% faster than four wavefronts of 4 x 4 blocks.
template <int WC>
struct SkShape {
  static constexpr int waves = 2 * WC, threads = 64 * waves;
  static constexpr int TC = 8 / WC;  // 16 x 16 blocks per wavefront, columns
};
constexpr int kSkWC = 4;

// Tile t over k in [kbeg, kend) into acc (the whole workgroup takes part).
// VEC: 16-byte loads (rows of X and w 16-byte aligned, k range even);
// otherwise element loads, any alignment and length.
template <int WC, bool VEC = true>
__device__ __forceinline__ void sk_tile(int mm, const double* __restrict__ X, long ldx,
                                        const double* __restrict__ w, int t, int kbeg, int kend,
                                        sk4 (&acc)[kSkT][SkShape<WC>::TC], bool active) {
  constexpr int NT = SkShape<WC>::threads, TC = SkShape<WC>::TC;
  constexpr int PPR = kSkKC / 2;
  constexpr int PAIRS = kSkBM * PPR / NT;
  __shared__ __attribute__((aligned(16))) double lds[2][2][kSkBM * kSkLS];
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * kSkBM, col0 = tj * kSkBM;
  const int nst = (kend - kbeg + kSkKC - 1) / kSkKC;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv / WC) * (16 * kSkT), wc0 = (wv % WC) * (16 * TC);
  double2 pa[PAIRS], pb[PAIRS], pw[PAIRS];
  auto gload = [&](int st) {
    const int kb = kbeg + st * kSkKC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + NT * it;
      const int row = p / PPR, k = kb + 2 * (p % PPR);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      if (VEC) {
        const int kc = min(k, kend - 2);
        pa[it] = *reinterpret_cast<const double2*>(X + ra * ldx + kc);
        pb[it] = *reinterpret_cast<const double2*>(X + rb * ldx + kc);
        pw[it] = *reinterpret_cast<const double2*>(w + kc);
      } else {
        // each element from its own column (clamped into the row; entries
        // beyond kend are zeroed when staged)
        const int k0 = min(k, kend - 1), k1 = min(k + 1, kend - 1);
        pa[it].x = X[ra * ldx + k0];
        pa[it].y = X[ra * ldx + k1];
        pb[it].x = X[rb * ldx + k0];
        pb[it].y = X[rb * ldx + k1];
        pw[it].x = w[k0];
        pw[it].y = w[k1];
      }
    }
  };
  auto sstore = [&](int buf, int st) {
    const int kb = kbeg + st * kSkKC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + NT * it;
      const int row = p / PPR, kk = 2 * (p % PPR), k = kb + kk;
      const bool va = row0 + row < mm, vb = col0 + row < mm;
      const bool v0 = k < kend, v1 = k + 1 < kend;
      double2 sa, sb;
      sa.x = (va && v0) ? pa[it].x * pw[it].x : 0.0;
      sa.y = (va && v1) ? pa[it].y * pw[it].y : 0.0;
      sb.x = (vb && v0) ? pb[it].x : 0.0;
      sb.y = (vb && v1) ? pb[it].y : 0.0;
      double* da = &lds[buf][0][row * kSkLS + kk];
      double* db = &lds[buf][1][row * kSkLS + kk];
      da[0] = sa.x;
      da[1] = sa.y;
      db[0] = sb.x;
      db[1] = sb.y;
    }
  };
  if (nst > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload(st + 1);
    if (active) {
      const double* la = lds[cur][0];
      const double* lb = lds[cur][1];
#pragma unroll
      for (int ks = 0; ks < kSkKC / 4; ++ks) {
        double a[kSkT], b[TC];
#pragma unroll
        for (int r = 0; r < kSkT; ++r) a[r] = la[(wr0 + 16 * r + li) * kSkLS + 4 * ks + lk];
#pragma unroll
        for (int c = 0; c < TC; ++c) b[c] = lb[(wc0 + 16 * c + li) * kSkLS + 4 * ks + lk];
#pragma unroll
        for (int r = 0; r < kSkT; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[c], acc[r][c], 0, 0, 0);
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1, st + 1);
    __syncthreads();
  }
}

// Batched normal matrices on the stream-K tile routine: LP = blockIdx.y,
// lower 128-tile blockIdx.x of M_i = A_i diag(d_i) A_i^T over the whole sum
// (no split).  A tile reads each of its two 128-row panels of A_i once, so
// an LP with m <= 128 reads its A once per operand and one with m <= 256
// three times, against nine times with 32-row tiles; element loads, since
// the rows of A_i need not be aligned or of even length.
__global__ __launch_bounds__(SkShape<kSkWC>::threads) void k_bsyrk_normal_sk(
    const BatchLP* __restrict__ lps, const int* __restrict__ go, const double* __restrict__ A,
    const double* __restrict__ d, double* __restrict__ Mpool) {
  constexpr int TC = SkShape<kSkWC>::TC;
  const int lp = blockIdx.y;
  if (!go[lp]) return;
  const BatchLP P = lps[lp];
  const int nt = (P.m + kSkBM - 1) / kSkBM, ntiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * kSkBM, col0 = tj * kSkBM;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv / kSkWC) * (16 * kSkT), wc0 = (wv % kSkWC) * (16 * TC);
  const bool active = !(ti == tj && wr0 + 16 * kSkT <= wc0);
  sk4 acc[kSkT][TC];
#pragma unroll
  for (int r = 0; r < kSkT; ++r)
#pragma unroll
    for (int c = 0; c < TC; ++c) acc[r][c] = sk4{0.0, 0.0, 0.0, 0.0};
  sk_tile<kSkWC, false>(P.m, A + P.a_off, P.n, d + P.vn, t, 0, P.n, acc, active);
  if (!active) return;
  double* C = Mpool + P.M_off;
#pragma unroll
  for (int r = 0; r < kSkT; ++r)
#pragma unroll
    for (int c = 0; c < TC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = row0 + wr0 + 16 * r + lk + 4 * v, gc = col0 + wc0 + 16 * c + li;
        if (gr < P.m && gc <= gr) C[(long)gr * P.ldm + gc] = acc[r][c][v];
      }
}

// Batched normal matrices on v_mfma_f64_16x16x4f64 (lane layout as in the
// stream-K routine above): lower BM-tile t of M_i = A_i diag(d_i) A_i^T over
// the whole sum, 2 x 2 wavefronts of (BM/2) x (BM/2), stages of KC along K
// through double-buffered LDS rows padded by two doubles.  BM = 32 (one
// 16 x 16 block per wavefront) or 64 (2 x 2 blocks); element loads, since
// the rows of A_i need not be aligned or of even length.  One-dimensional
// grid of T x count8 workgroups (T = lower tiles of the largest LP, count8
// = count rounded up to 8): workgroup b runs on XCD b % 8 and takes LP
// 8 (j / T) + b % 8, tile j % T with j = b / 8, so all tiles of an LP share
// one XCD's L2 and start together; they read the LP's A from that cache
// after its first pass.
// RHS: the diagonal tiles, which stage every row of A_i over the whole sum,
// also form the right-hand side rhs_i = b_i + A_i w_i of their rows (w_i the
// LP's d o r_d): each thread accumulates its staged elements times w in
// stage order, then the 16 threads of a row add their sums in a fixed
// butterfly order.
template <int BM, int KC>
constexpr int bsyrk16_lds_doubles() {
  return 2 * 2 * BM * (KC + 2);
}

// Lower tile t of LP P (the whole workgroup; t below the LP's tile count).
template <int BM, int KC, bool RHS>
__device__ __forceinline__ void bsyrk16_tile(const BatchLP& P, int t,
                                             const double* __restrict__ A,
                                             const double* __restrict__ d,
                                             double* __restrict__ Mpool,
                                             const double* __restrict__ wpool,
                                             const double* __restrict__ bpool,
                                             double* __restrict__ rhspool, double* lds_base) {
  constexpr int TB = BM / 32;             // 16 x 16 blocks per wavefront edge
  constexpr int LS = KC + 2;              // padded LDS row length
  constexpr int PPR = KC / 2;             // element pairs per row per stage
  constexpr int PAIRS = BM * PPR / 256;   // pairs per thread per operand
  static_assert(PAIRS >= 1 && BM * PPR % 256 == 0, "stage shape");
  double(*lds)[2][BM * LS] = reinterpret_cast<double(*)[2][BM * LS]>(lds_base);
  const int mm = P.m, K = P.n;
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  const double* __restrict__ X = A + P.a_off;
  const double* __restrict__ w = d + P.vn;
  const int nst = (K + KC - 1) / KC;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv >> 1) * (BM / 2), wc0 = (wv & 1) * (BM / 2);
  // the wavefront of a diagonal tile that lies wholly above the diagonal idles
  const bool active = !(ti == tj && wr0 + BM / 2 <= wc0);
  const bool diag = RHS && ti == tj;
  const double* __restrict__ wr = wpool + P.vn;
  sk4 acc[TB][TB];
#pragma unroll
  for (int r = 0; r < TB; ++r)
#pragma unroll
    for (int c = 0; c < TB; ++c) acc[r][c] = sk4{0.0, 0.0, 0.0, 0.0};
  double2 pa[PAIRS], pb[PAIRS], pw[PAIRS], pr[PAIRS];
  double racc[PAIRS];
#pragma unroll
  for (int it = 0; it < PAIRS; ++it) racc[it] = 0.0;
  auto gload = [&](int st) {
    const int kb = st * KC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / PPR, k = kb + 2 * (p % PPR);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      const int k0 = min(k, K - 1), k1 = min(k + 1, K - 1);
      pa[it].x = X[ra * K + k0];
      pa[it].y = X[ra * K + k1];
      pb[it].x = X[rb * K + k0];
      pb[it].y = X[rb * K + k1];
      pw[it].x = w[k0];
      pw[it].y = w[k1];
      if (diag) {
        pr[it].x = wr[k0];
        pr[it].y = wr[k1];
      }
    }
  };
  auto sstore = [&](int buf, int st) {
    const int kb = st * KC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / PPR, kk = 2 * (p % PPR), k = kb + kk;
      const bool va = row0 + row < mm, vb = col0 + row < mm;
      const bool v0 = k < K, v1 = k + 1 < K;
      if (diag) {
        racc[it] = fma(v0 ? pa[it].x : 0.0, pr[it].x, racc[it]);
        racc[it] = fma(v1 ? pa[it].y : 0.0, pr[it].y, racc[it]);
      }
      double2 sa, sb;
      sa.x = (va && v0) ? pa[it].x * pw[it].x : 0.0;
      sa.y = (va && v1) ? pa[it].y * pw[it].y : 0.0;
      sb.x = (vb && v0) ? pb[it].x : 0.0;
      sb.y = (vb && v1) ? pb[it].y : 0.0;
      *reinterpret_cast<double2*>(&lds[buf][0][row * LS + kk]) = sa;
      *reinterpret_cast<double2*>(&lds[buf][1][row * LS + kk]) = sb;
    }
  };
  if (nst > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) gload(st + 1);
    if (active) {
      const double* la = lds[cur][0];
      const double* lb = lds[cur][1];
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        double a[TB], bb[TB];
#pragma unroll
        for (int r = 0; r < TB; ++r) a[r] = la[(wr0 + 16 * r + li) * LS + 4 * ks + lk];
#pragma unroll
        for (int c = 0; c < TB; ++c) bb[c] = lb[(wc0 + 16 * c + li) * LS + 4 * ks + lk];
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
          for (int c = 0; c < TB; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], bb[c], acc[r][c], 0, 0, 0);
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1, st + 1);
    __syncthreads();
  }
  if (diag) {
    // the PPR = 16 threads of a row are 16 aligned consecutive lanes
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      double v = racc[it];
#pragma unroll
      for (int o = PPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      const int p = tid + 256 * it, gr = row0 + p / PPR;
      if (p % PPR == 0 && gr < mm) rhspool[P.vm + gr] = bpool[P.vm + gr] + v;
    }
  }
  if (!active) return;
  double* C = Mpool + P.M_off;
#pragma unroll
  for (int r = 0; r < TB; ++r)
#pragma unroll
    for (int c = 0; c < TB; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = row0 + wr0 + 16 * r + lk + 4 * v, gc = col0 + wc0 + 16 * c + li;
        if (gr < mm && gc <= gr) C[(long)gr * P.ldm + gc] = acc[r][c][v];
      }
}

template <int BM, int KC, bool RHS>
__global__ __launch_bounds__(256) void k_bsyrk_normal16(
    const BatchLP* __restrict__ lps, const int* __restrict__ go, const double* __restrict__ A,
    const double* __restrict__ d, double* __restrict__ Mpool, int count, int T,
    const double* __restrict__ wpool, const double* __restrict__ bpool,
    double* __restrict__ rhspool) {
  __shared__ __attribute__((aligned(16))) double lds[bsyrk16_lds_doubles<BM, KC>()];
  const int b = blockIdx.x, j = b >> 3;
  const int lp = (j / T) * 8 + (b & 7), t = j % T;
  if (lp >= count || !go[lp]) return;
  const BatchLP P = lps[lp];
  const int nt = (P.m + BM - 1) / BM;
  if (t >= nt * (nt + 1) / 2) return;
  bsyrk16_tile<BM, KC, RHS>(P, t, A, d, Mpool, wpool, bpool, rhspool, lds);
}

// Per-LP tile edge: 64 (intensity) for LPs with m > kBsyrkSmall, 32 (less
// padding) for the others; with m at most 4 kBsyrkSmall an LP of either kind
// has at most 10 lower tiles, so the grid (T tiles per LP, mapped to XCDs
// as above) carries few idle workgroups.
constexpr int kBsyrkSmall = 128;
template <bool RHS>
__global__ __launch_bounds__(256) void k_bsyrk_normal_hy(
    const BatchLP* __restrict__ lps, const int* __restrict__ go, const double* __restrict__ A,
    const double* __restrict__ d, double* __restrict__ Mpool, int count, int T,
    const double* __restrict__ wpool, const double* __restrict__ bpool,
    double* __restrict__ rhspool) {
  constexpr int L32 = bsyrk16_lds_doubles<32, 32>(), L64 = bsyrk16_lds_doubles<64, 16>();
  __shared__ __attribute__((aligned(16))) double lds[L32 > L64 ? L32 : L64];
  const int b = blockIdx.x, j = b >> 3;
  const int lp = (j / T) * 8 + (b & 7), t = j % T;
  if (lp >= count || !go[lp]) return;
  const BatchLP P = lps[lp];
  const bool big = P.m > kBsyrkSmall;
  const int bm = big ? 64 : 32;
  const int nt = (P.m + bm - 1) / bm;
  if (t >= nt * (nt + 1) / 2) return;
  if (big) bsyrk16_tile<64, 16, RHS>(P, t, A, d, Mpool, wpool, bpool, rhspool, lds);
  else bsyrk16_tile<32, 32, RHS>(P, t, A, d, Mpool, wpool, bpool, rhspool, lds);
}

// C (lower, ldc) = X diag(w) X^T; X rows 16-byte aligned, K even.
// part: kSkGroups * 2 partial tiles, then one arrival counter per tile
// (zero on entry; every counter is back at zero when the launch ends).
template <int WC>
__global__ __launch_bounds__(SkShape<WC>::threads) void k_syrk_sk(
    int mm, int K, const double* __restrict__ X, long ldx, const double* __restrict__ w,
    double* __restrict__ C, long ldc, int ntiles, int G, double* __restrict__ part) {
  // G <= kSkGroups workgroups, at most one per unit of work, so that every
  // range is non-empty (a tile's counter expects one arrival per range that
  // meets it); the XCD remap needs G to be a multiple of 8
  constexpr int BM = kSkBM, TC = SkShape<WC>::TC, NQ = kSkT * TC;
  const int S = (K + kSkKC - 1) / kSkKC;
  const long W = (long)ntiles * S;
  const int g = (G % 8 == 0) ? (int)((blockIdx.x & 7) * (G / 8) + (blockIdx.x >> 3))
                             : (int)blockIdx.x;
  auto bnd = [&](long gg) { return gg * W / G; };
  const long b0 = bnd(g), b1 = bnd(g + 1);
  int* cnt = reinterpret_cast<int*>(part + (long)kSkGroups * 2 * BM * BM);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr0 = (wv / WC) * (16 * kSkT), wc0 = (wv % WC) * (16 * TC);
  __shared__ int s_last;
  for (long it = b0; it < b1;) {
    const int t = (int)(it / S), s0 = (int)(it % S);
    const int s1 = (int)min((long)S, s0 + (b1 - it));
    int ti, tj;
    tile_coords(t, ti, tj);
    const int row0 = ti * BM, col0 = tj * BM;
    // wavefronts of a diagonal tile whose block lies above the diagonal idle
    const bool active = !(ti == tj && wr0 + 16 * kSkT <= wc0);
    sk4 acc[kSkT][TC];
#pragma unroll
    for (int r = 0; r < kSkT; ++r)
#pragma unroll
      for (int c = 0; c < TC; ++c) acc[r][c] = sk4{0.0, 0.0, 0.0, 0.0};
    sk_tile<WC>(mm, X, ldx, w, t, s0 * kSkKC, min(K, s1 * kSkKC), acc, active);
    const bool whole = (s0 == 0 && s1 == S);
    if (whole) {
      if (active) {
#pragma unroll
        for (int r = 0; r < kSkT; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int gr = row0 + wr0 + 16 * r + lk + 4 * v, gc = col0 + wc0 + 16 * c + li;
              if (gr < mm && gc <= gr) C[(long)gr * ldc + gc] = acc[r][c][v];
            }
      }
    } else {
      // partial tile in register order (lane-contiguous, so both the store and
      // the reducer's loads are coalesced): element (q = r TC + c, v) of
      // lane l of wavefront wv at ((wv * NQ + q) * 64 + l) * 4 + v
      double* P = part + ((long)g * 2 + (it == b0 ? 0 : 1)) * (BM * BM);
      if (active) {
#pragma unroll
        for (int r = 0; r < kSkT; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c)
            *reinterpret_cast<sk4*>(P + ((wv * NQ + r * TC + c) * 64 + lane) * 4) = acc[r][c];
      }
      // the workgroups whose ranges meet tile t
      const long xs = (long)t * S, xe = xs + S - 1;
      long glo = xs * G / W, ghi = xe * G / W;
      while (bnd(glo) > xs) --glo;
      while (bnd(glo + 1) <= xs) ++glo;
      while (bnd(ghi) > xe) --ghi;
      while (bnd(ghi + 1) <= xe) ++ghi;
      const int nseg = (int)(ghi - glo + 1);
      // One device-scope release / acquire per workgroup, by thread 0 (the
      // counter update), not one per thread: each is a writeback (and
      // invalidate) of the whole L2 of its XCD, which by then holds most
      // of the partial tiles, and hundreds of them at the end of the
      // launch cost more than the tile work.  Every wavefront first waits
      // for its own partial stores; the barriers carry the ordering from
      // and to the other wavefronts of the workgroup.
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (tid == 0) {
        const int prev = __hip_atomic_fetch_add(&cnt[t], 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == nseg - 1);
        if (s_last) __hip_atomic_store(&cnt[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (s_last && active) {
        // sum of the segments in workgroup order; this workgroup's own
        // segment is still in registers
        sk4 tot[kSkT][TC];
#pragma unroll
        for (int r = 0; r < kSkT; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c) tot[r][c] = sk4{0.0, 0.0, 0.0, 0.0};
        for (long gg = glo; gg <= ghi; ++gg) {
          if (gg == g) {
#pragma unroll
            for (int r = 0; r < kSkT; ++r)
#pragma unroll
              for (int c = 0; c < TC; ++c) tot[r][c] += acc[r][c];
          } else {
            // slot 0 when tile t is where workgroup gg's range starts
            const int sl = (bnd(gg) / S == t) ? 0 : 1;
            const double* Q = part + (gg * 2 + sl) * (BM * BM);
            sk4 pv[kSkT][TC];
#pragma unroll
            for (int r = 0; r < kSkT; ++r)
#pragma unroll
              for (int c = 0; c < TC; ++c)
                pv[r][c] = *reinterpret_cast<const sk4*>(Q + ((wv * NQ + r * TC + c) * 64 + lane) * 4);
#pragma unroll
            for (int r = 0; r < kSkT; ++r)
#pragma unroll
              for (int c = 0; c < TC; ++c) tot[r][c] += pv[r][c];
          }
        }
#pragma unroll
        for (int r = 0; r < kSkT; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int gr = row0 + wr0 + 16 * r + lk + 4 * v, gc = col0 + wc0 + 16 * c + li;
              if (gr < mm && gc <= gr) C[(long)gr * ldc + gc] = tot[r][c][v];
            }
      }
      __syncthreads();
    }
    it += s1 - s0;
  }
}

}  // namespace

size_t syrk_part_elems(int mm, int tile, int splits) {
  if (tile == 0) {
    // stream-K: two partial tiles per workgroup, then the tile counters
    const long nt = cdiv(mm, kSkBM);
    const size_t ntiles = (size_t)(nt * (nt + 1) / 2);
    return (size_t)kSkGroups * 2 * kSkBM * kSkBM + (ntiles + 1) / 2;
  }
  if (splits <= 1) return 0;
  const long nt = cdiv(mm, tile);
  const size_t ntiles = (size_t)(nt * (nt + 1) / 2);
  // partial tiles, then one arrival counter (int) per tile
  return (size_t)splits * ntiles * (size_t)tile * tile + (ntiles + 1) / 2;
}

void syrk_choose(int mm, int K, int* tile, int* splits) {
  // Large problems: the stream-K kernel (tile 0).
  if (mm >= 512 && K >= 1024) {
    *tile = 0;
    *splits = 1;
    return;
  }
  // Otherwise split-K: 128 x 128 tiles for large outputs, 64 x 64 for small.
  const int t = mm >= 1024 ? 128 : 64;
  const long nt = cdiv(mm, t);
  const long ntiles = nt * (nt + 1) / 2;
  // Split the sum over j until about three rounds of workgroups cover the 256
  // CUs, keeping at least 256 of K per split (more splits fill the last round
  // better but add partial-tile traffic; paper_1502_03543_amd/autotune.py
  // measures the best count per shape).
  static const int kSplits[] = {1, 2, 3, 4, 6, 8, 12, 16};
  int s = 1;
  for (int c : kSplits) {
    if ((long)K / c < 256) break;
    s = c;
    if (ntiles * c >= 768) break;
  }
  *tile = t;
  *splits = s;
}

void launch_syrk_f64(hipStream_t st, int mm, int K, const double* X, long ldx, const double* w,
                     double* C, long ldc, bool sub, int tile, int splits, double* part,
                     hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (mm <= 0) return;
  const bool vec = ((ldx & 1) == 0) && (((uintptr_t)X & 15) == 0) && ((K & 1) == 0) &&
                   (!w || (((uintptr_t)w & 15) == 0));
  if (tile == 0) {
    if (w && !sub && vec && part && K >= 2) {
      const int nt = cdiv(mm, kSkBM);
      const int ntiles = nt * (nt + 1) / 2;
      launch_fill_i32(st, reinterpret_cast<int*>(part + (size_t)kSkGroups * 2 * kSkBM * kSkBM), 0,
                      ntiles);
      if (ev_begin) (void)hipEventRecord(ev_begin, st);
      const long work = (long)ntiles * cdiv(K, kSkKC);
      int G = kSkGroups;
      if (work < G) G = work >= 8 ? (int)(work / 8 * 8) : (int)work;
      hipLaunchKernelGGL(k_syrk_sk<kSkWC>, dim3(G), dim3(SkShape<kSkWC>::threads), 0, st, mm, K,
                         X, ldx, w, C, ldc, ntiles, G, part);
      if (ev_end) (void)hipEventRecord(ev_end, st);
      return;
    }
    // operands the stream-K kernel does not take: one 64-tile pass
    tile = 64;
    splits = 1;
  }
  const int nt = cdiv(mm, tile);
  const int ntiles = nt * (nt + 1) / 2;
  const int per_xcd = cdiv(ntiles, 8);
  const int kc = tile == 128 ? kKC128 : kKC64;
  int kchunk = cdiv(cdiv(K, splits), kc) * kc;
  if (splits <= 1 || !part) {
    splits = 1;
    kchunk = K;
    part = nullptr;
  }
  if (part) {
    // arrival counters of the split tiles start at zero
    launch_fill_i32(st, reinterpret_cast<int*>(part + (size_t)splits * ntiles * tile * tile), 0,
                    ntiles);
  }
  dim3 grid(8 * per_xcd, splits);
  if (ev_begin) (void)hipEventRecord(ev_begin, st);
#define PDAS_SYRK(R_, Q_, KC_, S_, V_)                                                        \
  hipLaunchKernelGGL((k_syrk_f64<R_, Q_, KC_, S_, V_>), grid, dim3(256), 0, st, mm, K, X, ldx, \
                     w, C, ldc, (int)sub, ntiles, per_xcd, kchunk, part)
  if (tile == 128) {
    if (w) {
      if (vec) PDAS_SYRK(16, 4, kKC128, true, true);
      else PDAS_SYRK(16, 4, kKC128, true, false);
    } else {
      if (vec) PDAS_SYRK(16, 4, kKC128, false, true);
      else PDAS_SYRK(16, 4, kKC128, false, false);
    }
  } else {
    if (w) {
      if (vec) PDAS_SYRK(8, 2, kKC64, true, true);
      else PDAS_SYRK(8, 2, kKC64, true, false);
    } else {
      if (vec) PDAS_SYRK(8, 2, kKC64, false, true);
      else PDAS_SYRK(8, 2, kKC64, false, false);
    }
  }
#undef PDAS_SYRK
  if (ev_end) (void)hipEventRecord(ev_end, st);
}

size_t syrk_part_elems_f32(int mm, int splits) {
  if (splits <= 1) return 0;
  const long nt = cdiv(mm, 128);
  return (size_t)splits * (size_t)(nt * (nt + 1) / 2) * 128u * 128u;
}

void syrk_choose_f32(int mm, int K, int* splits) {
  const long nt = cdiv(mm, 128);
  const long ntiles = nt * (nt + 1) / 2;
  int s = 1;
  while (ntiles * s < 512 && (long)K / (2 * s) >= 512) s *= 2;
  *splits = s;
}

bool launch_syrk_f32(hipStream_t st, int mm, int K, const float* X, long ldx, const float* w,
                     float* C, long ldc, bool sub, int splits, float* part, hipEvent_t ev_begin,
                     hipEvent_t ev_end) {
  if (mm <= 0) return true;
  // 16-byte loads need 4-aligned K and rows
  if ((K & 3) || (ldx & 3) || ((uintptr_t)X & 15) || (w && ((uintptr_t)w & 15))) return false;
  constexpr int BM = 128, KC = 32;
  const int nt = cdiv(mm, BM);
  const int ntiles = nt * (nt + 1) / 2;
  const int per_xcd = cdiv(ntiles, 8);
  int kchunk = cdiv(cdiv(K, splits), KC) * KC;
  if (splits <= 1 || !part) {
    splits = 1;
    kchunk = K;
    part = nullptr;
  }
  dim3 grid(8 * per_xcd, splits);
  if (ev_begin) (void)hipEventRecord(ev_begin, st);
  if (w)
    hipLaunchKernelGGL((k_syrk_f32<4, KC, true>), grid, dim3(256), 0, st, mm, K, X, ldx, w, C,
                       ldc, (int)sub, ntiles, per_xcd, kchunk, part);
  else
    hipLaunchKernelGGL((k_syrk_f32<4, KC, false>), grid, dim3(256), 0, st, mm, K, X, ldx, w, C,
                       ldc, (int)sub, ntiles, per_xcd, kchunk, part);
  if (ev_end) (void)hipEventRecord(ev_end, st);
  if (part)
    hipLaunchKernelGGL(k_syrk_reduce_f32<BM>, dim3(ntiles), dim3(256), 0, st, mm, C, ldc,
                       (int)sub, ntiles, splits, part);
  return true;
}

bool launch_bsyrk_normal(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                         const int* go, const double* A, const double* d, double* Mpool,
                         const double* w, const double* b, double* rhs) {
  if (tile == 0) {
    const int n64 = cdiv(max_m, 64), n32 = cdiv(std::min(max_m, kBsyrkSmall), 32);
    const int T = std::max(n64 * (n64 + 1) / 2, n32 * (n32 + 1) / 2);
    const dim3 grid(T * 8 * cdiv(count, 8));
    if (rhs)
      hipLaunchKernelGGL(k_bsyrk_normal_hy<true>, grid, dim3(256), 0, st, lps, go, A, d, Mpool,
                         count, T, w, b, rhs);
    else
      hipLaunchKernelGGL(k_bsyrk_normal_hy<false>, grid, dim3(256), 0, st, lps, go, A, d, Mpool,
                         count, T, w, b, rhs);
    return rhs != nullptr;
  }
  const int nt = cdiv(max_m, tile);
  if (tile == 128) {
    hipLaunchKernelGGL(k_bsyrk_normal_sk, dim3(nt * (nt + 1) / 2, count),
                       dim3(SkShape<kSkWC>::threads), 0, st, lps, go, A, d, Mpool);
    return false;
  }
  const int T = nt * (nt + 1) / 2;
  const dim3 grid(T * 8 * cdiv(count, 8));
  if (rhs) {
    if (tile == 32)
      hipLaunchKernelGGL((k_bsyrk_normal16<32, 32, true>), grid, dim3(256), 0, st, lps, go, A, d,
                         Mpool, count, T, w, b, rhs);
    else
      hipLaunchKernelGGL((k_bsyrk_normal16<64, 16, true>), grid, dim3(256), 0, st, lps, go, A, d,
                         Mpool, count, T, w, b, rhs);
    return true;
  }
  if (tile == 32)
    hipLaunchKernelGGL((k_bsyrk_normal16<32, 32, false>), grid, dim3(256), 0, st, lps, go, A, d,
                       Mpool, count, T, w, b, rhs);
  else
    hipLaunchKernelGGL((k_bsyrk_normal16<64, 16, false>), grid, dim3(256), 0, st, lps, go, A, d,
                       Mpool, count, T, w, b, rhs);
  return false;
}

void launch_bsyrk_trailing(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                           const int* go, double* Mpool, int p) {
  const int mm = max_m - p - 64;
  if (mm <= 0) return;
  if (tile == 0) tile = 32;  // the library's choice beside per-LP normal-matrix tiles
  if (tile > 64) tile = 64;  // the K = 64 updates keep 64-row tiles
  const int nt = cdiv(mm, tile);
  if (tile == 32)
    hipLaunchKernelGGL(k_bsyrk_trailing<32>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, Mpool, p);
  else
    hipLaunchKernelGGL(k_bsyrk_trailing<64>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, Mpool, p);
}

void launch_bsyrk_normal_f32(hipStream_t st, int count, int max_m, int tile, const BatchLP* lps,
                             const int* go, const float* A32, const float* sd32, float* M32) {
  if (tile == 0 || tile > 64) tile = 64;
  const int nt = cdiv(max_m, tile);
  if (tile == 32)
    hipLaunchKernelGGL(k_bsyrk_normal_f32<1>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, A32, sd32, M32);
  else
    hipLaunchKernelGGL(k_bsyrk_normal_f32<2>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, A32, sd32, M32);
}

void launch_bsyrk_trailing_f32(hipStream_t st, int count, int max_m, int tile,
                               const BatchLP* lps, const int* go, float* M32, int p) {
  const int mm = max_m - p - 64;
  if (mm <= 0) return;
  if (tile == 0 || tile > 64) tile = 64;
  const int nt = cdiv(mm, tile);
  if (tile == 32)
    hipLaunchKernelGGL(k_bsyrk_trailing_f32<1>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, M32, p);
  else
    hipLaunchKernelGGL(k_bsyrk_trailing_f32<2>, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st,
                       lps, go, M32, p);
}

}  // namespace pdas
