// Normal matrix M = A D A^T of the Section 5 normal equations, on the FP64
// matrix cores of gfx950, and the same kernel in subtract mode for the
// Cholesky trailing update (C -= L21 L21^T).
//
// Instruction: v_mfma_f64_4x4x4_4b (four independent 4x4x4 products per
// wavefront; it sustains close to the FP64 matrix peak on gfx950, unlike the
// 16x16x4 form).  Lane l = x + 4*blk + 16*y holds
//   A operand: rowop[i = x][k = y] of block blk,
//   B operand: colop[j = x][k = y] of block blk,
//   D result : C[i = y][j = x] of block blk.
// A wavefront register-blocks a (4R) x (16Q) output: the A operand carries 4
// rows (identical across the 4 blocks), the B operand 16 columns (4 per
// block), so each instruction produces a 4 x 16 slab for K = 4.
//
// Workgroup: 256 threads = 2 x 2 wavefronts; tile BM = 8R rows by BN = 32Q
// columns (square).  Only tiles on or below the diagonal are launched.  Both
// operands stream through double-buffered LDS in chunks of 16 along K, laid
// out so that every LDS read of a wavefront is lane-linear (B) or a 4-way
// broadcast (A).  The diagonal weight d is applied to the row operand while
// it is staged.  Split-K writes per-split partial tiles that an ordered
// second pass sums, so results do not depend on scheduling.
#include <cmath>

#include "pdas_internal.h"

namespace pdas {
namespace {

constexpr int KC = 16;  // K per LDS stage

__device__ inline void tile_coords(int t, int& ti, int& tj) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

// LDS index of element (row, k) of a BM x KC stage buffer.
template <int BM>
__device__ inline int lidx(int row, int k) {
  return (((k >> 2) * (BM / 16) + (row >> 4)) << 6) + ((k & 3) << 4) + (row & 15);
}

template <int R, int Q>
__global__ __launch_bounds__(256) void k_syrk_f64(int mm, int K, const double* __restrict__ X,
                                                  long ldx, const double* __restrict__ w,
                                                  double* __restrict__ C, long ldc, int sub,
                                                  int ntiles, int per_xcd, int kchunk,
                                                  double* __restrict__ part) {
  constexpr int BM = 8 * R;
  static_assert(BM == 32 * Q, "square tiles");
  constexpr int PAIRS = BM * KC / 2 / 256;  // 16-byte pairs per thread per operand
  __shared__ double lds[2][2][BM * KC];     // [stage][operand: 0 rows, 1 cols]

  // XCD-aware order: consecutive tiles (sharing row panels) on one XCD.
  const int b = blockIdx.x;
  const int t = (b & 7) * per_xcd + (b >> 3);
  if (t >= ntiles) return;
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  const int split = blockIdx.y;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nst = (kend - kbeg + KC - 1) / KC;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int x = lane & 3, blk = (lane >> 2) & 3, y = lane >> 4;
  const int wr0 = (wv >> 1) * (4 * R), wc0 = (wv & 1) * (16 * Q);
  // wavefronts of a diagonal tile whose block lies strictly above the diagonal idle
  const bool active = !(ti == tj && wr0 + 4 * R <= wc0);
  const bool vec = ((ldx & 1) == 0) && ((((uintptr_t)X) & 15) == 0);

  double acc[R][Q];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[r][q] = 0.0;

  double pa[PAIRS][2], pb[PAIRS][2];
  auto gload = [&](int st) {
    const int kb = kbeg + st * KC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p >> 3, k = kb + ((p & 7) << 1);
      const int ra = row0 + row, rb = col0 + row;
      double a0 = 0, a1 = 0, b0 = 0, b1 = 0;
      if (vec && k + 1 < kend) {
        if (ra < mm) {
          const double2 v = *reinterpret_cast<const double2*>(X + (long)ra * ldx + k);
          a0 = v.x;
          a1 = v.y;
        }
        if (rb < mm) {
          const double2 v = *reinterpret_cast<const double2*>(X + (long)rb * ldx + k);
          b0 = v.x;
          b1 = v.y;
        }
      } else {
        if (ra < mm && k < kend) a0 = X[(long)ra * ldx + k];
        if (ra < mm && k + 1 < kend) a1 = X[(long)ra * ldx + k + 1];
        if (rb < mm && k < kend) b0 = X[(long)rb * ldx + k];
        if (rb < mm && k + 1 < kend) b1 = X[(long)rb * ldx + k + 1];
      }
      if (w) {
        if (k < kend) a0 *= w[k];
        if (k + 1 < kend) a1 *= w[k + 1];
      }
      pa[it][0] = a0;
      pa[it][1] = a1;
      pb[it][0] = b0;
      pb[it][1] = b1;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p >> 3, k = (p & 7) << 1;
      lds[buf][0][lidx<BM>(row, k)] = pa[it][0];
      lds[buf][0][lidx<BM>(row, k + 1)] = pa[it][1];
      lds[buf][1][lidx<BM>(row, k)] = pb[it][0];
      lds[buf][1][lidx<BM>(row, k + 1)] = pb[it][1];
    }
  };

  if (nst > 0) {
    gload(0);
    sstore(0);
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
        double bq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = wc0 + 16 * q + 4 * blk + x;
          bq[q] = lb[lidx<BM>(c, 4 * ks + y)];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double av = la[lidx<BM>(wr0 + 4 * r + x, 4 * ks + y)];
#pragma unroll
          for (int q = 0; q < Q; ++q)
            acc[r][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bq[q], acc[r][q], 0, 0, 0);
        }
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1);
    __syncthreads();
  }

  if (!active) return;
  if (part) {
    double* P = part + ((long)split * ntiles + t) * (BM * BM);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int lr = wr0 + 4 * r + y, lc = wc0 + 16 * q + 4 * blk + x;
        P[lr * BM + lc] = acc[r][q];
      }
    return;
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int gr = row0 + wr0 + 4 * r + y, gc = col0 + wc0 + 16 * q + 4 * blk + x;
      if (gr < mm && gc <= gr) {
        double* cp = C + (long)gr * ldc + gc;
        *cp = sub ? (*cp - acc[r][q]) : acc[r][q];
      }
    }
}

// Ordered sum of split-K partial tiles into C (lower part only).
template <int BM>
__global__ __launch_bounds__(256) void k_syrk_reduce(int mm, double* __restrict__ C, long ldc,
                                                     int sub, int ntiles, int splits,
                                                     const double* __restrict__ part) {
  const int t = blockIdx.x;
  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  for (int e = threadIdx.x; e < BM * BM; e += 256) {
    const int lr = e / BM, lc = e % BM;
    const int gr = row0 + lr, gc = col0 + lc;
    if (gr >= mm || gc > gr) continue;
    double v = 0;
    for (int s = 0; s < splits; ++s) v += part[((long)s * ntiles + t) * (BM * BM) + e];
    double* cp = C + (long)gr * ldc + gc;
    *cp = sub ? (*cp - v) : v;
  }
}

}  // namespace

size_t syrk_part_elems(int mm, int tile, int splits) {
  if (splits <= 1) return 0;
  const long nt = cdiv(mm, tile);
  return (size_t)splits * (size_t)(nt * (nt + 1) / 2) * (size_t)tile * tile;
}

void syrk_choose(int mm, int K, int* tile, int* splits) {
  // Large outputs: 128 x 128 tiles; small outputs: 64 x 64 for parallelism.
  const int t = mm >= 1024 ? 128 : 64;
  const long nt = cdiv(mm, t);
  const long ntiles = nt * (nt + 1) / 2;
  int s = 1;
  // split K until there are enough workgroups to cover the 256 CUs twice,
  // keeping at least 256 of K per split.
  while (ntiles * s < 512 && (long)K / (2 * s) >= 256) s *= 2;
  *tile = t;
  *splits = s;
}

void launch_syrk_f64(hipStream_t st, int mm, int K, const double* X, long ldx, const double* w,
                     double* C, long ldc, bool sub, int tile, int splits, double* part,
                     hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (mm <= 0) return;
  const int nt = cdiv(mm, tile);
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
  if (tile == 128)
    hipLaunchKernelGGL((k_syrk_f64<16, 4>), grid, dim3(256), 0, st, mm, K, X, ldx, w, C, ldc,
                       (int)sub, ntiles, per_xcd, kchunk, part);
  else
    hipLaunchKernelGGL((k_syrk_f64<8, 2>), grid, dim3(256), 0, st, mm, K, X, ldx, w, C, ldc,
                       (int)sub, ntiles, per_xcd, kchunk, part);
  if (ev_end) (void)hipEventRecord(ev_end, st);
  if (part) {
    if (tile == 128)
      hipLaunchKernelGGL(k_syrk_reduce<128>, dim3(ntiles), dim3(256), 0, st, mm, C, ldc,
                         (int)sub, ntiles, splits, part);
    else
      hipLaunchKernelGGL(k_syrk_reduce<64>, dim3(ntiles), dim3(256), 0, st, mm, C, ldc,
                         (int)sub, ntiles, splits, part);
  }
}

}  // namespace pdas
