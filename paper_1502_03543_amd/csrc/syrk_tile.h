// Normal-matrix / trailing-update tile routine shared by the normal-matrix
// kernels and the fused Cholesky step (device code, included by both).
//
// Instruction: v_mfma_f64_4x4x4_4b (four independent 4x4x4 products per
// wavefront).  Lane l = x + 4*blk + 16*y holds
//   A operand: rowop[i = x][k = y] of block blk,
//   B operand: colop[j = x][k = y] of block blk,
//   D result : C[i = y][j = x] of block blk.
// A wavefront register-blocks a (4R) x (16Q) output: the A operand carries 4
// rows (identical across the 4 blocks), the B operand 16 columns (4 per
// block), so each instruction produces a 4 x 16 slab for K = 4.
//
// Workgroup: 256 threads = 2 x 2 wavefronts; tile BM = 8R rows by BN = 32Q
// columns (square).  Only tiles on or below the diagonal are launched.  Both
// operands stream through double-buffered LDS in stages of KC along K, row by
// row with a padded row length of KC + 4 doubles and 16-byte stage stores
// (a blocked layout of 4 k by 16 rows made every stage write a 16-way bank
// conflict).  Global loads for the next stage are issued before the MFMA
// work of the current one and consumed only when they are stored to LDS, so
// they stay in flight during the matrix work.  The diagonal weight d is
// applied to the row operand while it is staged.
#pragma once

#include "pdas_internal.h"

namespace pdas {
namespace {

__device__ inline void tile_coords(int t, int& ti, int& tj) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

// LDS index of element (row, k) of a BM x KC stage buffer: blocks of 4 k by
// 16 rows, so a wavefront's operand read is lane-linear.
template <int BM>
__device__ inline int lidx(int row, int k) {
  return (((k >> 2) * (BM / 16) + (row >> 4)) << 6) + ((k & 3) << 4) + (row & 15);
}

// R, Q: wavefront tile (4R) x (16Q); KC: K per stage; SCALE: multiply the row
// operand by w[k] while staging; VEC: 16-byte loads (X rows and w 16-byte
// aligned, K even).
// One lower tile t (linear index over the lower triangle of tiles) of one
// K split; the whole workgroup takes part.
template <int R, int Q, int KC, bool SCALE, bool VEC>
__device__ __forceinline__ void syrk_f64_tile(int mm, int K, const double* __restrict__ X,
                                              long ldx, const double* __restrict__ w,
                                              double* __restrict__ C, long ldc, int sub, int t,
                                              int ntiles, int split, int nsplit, int kchunk,
                                              double* __restrict__ part, double2* lds_base) {
  constexpr int BM = 8 * R;
  static_assert(BM == 32 * Q, "square tiles");
  constexpr int PPR = KC / 2;               // element pairs per row per stage
  constexpr int PAIRS = BM * PPR / 256;     // pairs per thread per operand
  constexpr int LS = KC + 4;                // padded LDS row length
  // [stage][operand: 0 rows, 1 cols] stage buffers in the caller's LDS
  double2(*lds2)[2][BM * LS / 2] = reinterpret_cast<double2(*)[2][BM * LS / 2]>(lds_base);

  int ti, tj;
  tile_coords(t, ti, tj);
  const int row0 = ti * BM, col0 = tj * BM;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int nst = (kend - kbeg + KC - 1) / KC;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int x = lane & 3, blk = (lane >> 2) & 3, y = lane >> 4;
  const int wr0 = (wv >> 1) * (4 * R), wc0 = (wv & 1) * (16 * Q);
  // wavefronts of a diagonal tile whose block lies strictly above the diagonal idle
  const bool active = !(ti == tj && wr0 + 4 * R <= wc0);

  double acc[R][Q];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[r][q] = 0.0;
  // In subtract mode without split the C values are loaded now, so their
  // latency overlaps the operand stream instead of following it.
  double cpre[R][Q];
  if (sub && !part) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int gr = min(row0 + wr0 + 4 * r + y, mm - 1);
        const int gc = min(col0 + wc0 + 16 * q + 4 * blk + x, gr);
        cpre[r][q] = active ? C[(long)gr * ldc + gc] : 0.0;
      }
  }

  // Staging registers.  Every load address is clamped into the valid range,
  // so the loads need no branches; elements outside the tile or the K range
  // are zeroed when the stage is stored to LDS.  Nothing consumes the loaded
  // values before the store, so they stay in flight during the MFMA work.
  double2 pa[PAIRS], pb[PAIRS], pw[PAIRS];
  auto gload = [&](int st) {
    const int kb = kbeg + st * KC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / PPR, k = kb + 2 * (p % PPR);
      const long ra = min(row0 + row, mm - 1), rb = min(col0 + row, mm - 1);
      if (VEC) {
        const int kc = min(k, kend - 2);
        pa[it] = *reinterpret_cast<const double2*>(X + ra * ldx + kc);
        pb[it] = *reinterpret_cast<const double2*>(X + rb * ldx + kc);
        if (SCALE) pw[it] = *reinterpret_cast<const double2*>(w + kc);
      } else {
        const int k0 = min(k, kend - 1), k1 = min(k + 1, kend - 1);
        pa[it].x = X[ra * ldx + k0];
        pa[it].y = X[ra * ldx + k1];
        pb[it].x = X[rb * ldx + k0];
        pb[it].y = X[rb * ldx + k1];
        if (SCALE) {
          pw[it].x = w[k0];
          pw[it].y = w[k1];
        }
      }
    }
  };
  auto sstore = [&](int buf, int st) {
    const int kb = kbeg + st * KC;
#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
      const int p = tid + 256 * it;
      const int row = p / PPR, kk = 2 * (p % PPR), k = kb + kk;
      const bool va = row0 + row < mm, vb = col0 + row < mm;
      const bool v0 = k < kend, v1 = k + 1 < kend;
      double a0 = pa[it].x, a1 = pa[it].y;
      if (SCALE) {
        a0 *= pw[it].x;
        a1 *= pw[it].y;
      }
      double2 sa, sb;
      sa.x = (va && v0) ? a0 : 0.0;
      sa.y = (va && v1) ? a1 : 0.0;
      sb.x = (vb && v0) ? pb[it].x : 0.0;
      sb.y = (vb && v1) ? pb[it].y : 0.0;
      lds2[buf][0][(row * LS + kk) / 2] = sa;
      lds2[buf][1][(row * LS + kk) / 2] = sb;
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
      const double* la = reinterpret_cast<const double*>(lds2[cur][0]);
      const double* lb = reinterpret_cast<const double*>(lds2[cur][1]);
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        double bq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = wc0 + 16 * q + 4 * blk + x;
          bq[q] = lb[c * LS + 4 * ks + y];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double av = la[(wr0 + 4 * r + x) * LS + 4 * ks + y];
#pragma unroll
          for (int q = 0; q < Q; ++q)
            acc[r][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bq[q], acc[r][q], 0, 0, 0);
        }
      }
    }
    if (st + 1 < nst) sstore(cur ^ 1, st + 1);
    __syncthreads();
  }

  if (part) {
    double* P = part + ((long)split * ntiles + t) * (BM * BM);
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int lr = wr0 + 4 * r + y, lc = wc0 + 16 * q + 4 * blk + x;
          P[lr * BM + lc] = acc[r][q];
        }
    }
    // The last split of this tile to arrive sums all partial tiles in split
    // order (so the result does not depend on which one arrives last).  The
    // only device-scope release / acquire is thread 0's counter update (each
    // one writes back / invalidates the XCD's whole L2): every wavefront
    // waits for its own stores, and the barriers order the other
    // wavefronts' accesses with it.
    __shared__ int s_last;
    int* cnt = reinterpret_cast<int*>(part + (long)nsplit * ntiles * (BM * BM));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      const int prev = __hip_atomic_fetch_add(&cnt[t], 1, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
      s_last = (prev == nsplit - 1);
      if (s_last) __hip_atomic_store(&cnt[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!s_last) return;
    for (int e = tid; e < BM * BM; e += 256) {
      const int lr = e / BM, lc = e % BM;
      const int gr = row0 + lr, gc = col0 + lc;
      if (gr >= mm || gc > gr) continue;
      double v = 0;
      for (int sp = 0; sp < nsplit; ++sp) v += part[((long)sp * ntiles + t) * (BM * BM) + e];
      double* cp = C + (long)gr * ldc + gc;
      *cp = sub ? (*cp - v) : v;
    }
    return;
  }
  if (!active) return;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int gr = row0 + wr0 + 4 * r + y, gc = col0 + wc0 + 16 * q + 4 * blk + x;
      if (gr < mm && gc <= gr) C[(long)gr * ldc + gc] = sub ? cpre[r][q] - acc[r][q] : acc[r][q];
    }
}

// LDS the tile routine needs (double2 elements), for stage length KC
template <int R, int KC>
constexpr int syrk_tile_lds2() {
  return 2 * 2 * (8 * R) * (KC + 4) / 2;
}

}  // namespace
}  // namespace pdas
