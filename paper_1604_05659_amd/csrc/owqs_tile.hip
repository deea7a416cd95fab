// owqs_tile.hip -- a run of commands in one pass over HBM (cache blocking in
// LDS).
//
// A group is a run of fused windows, E, X and Z steps at one live width n
// whose mixing slots (the slot a window or an X pairs amplitudes across) lie
// in a set T of k slots: the low kLowBits slots plus the group's mixing
// slots.  The vector splits into 2^(n-k) tiles of 2^k amplitudes (all values
// of the T bits, the other bits fixed); each workgroup loads a tile into LDS,
// applies every command of the group to it, and writes it back once.
// Diagonal factors (E, Z, and the index-parity signs of windows) read any
// bit: bits in T come from the local index, the others are constant over the
// tile and are evaluated once per tile.  Because T always holds the low five
// slots, every tile is made of 256-byte runs, so loads and stores coalesce.
//
// Probabilities (Eq. 13): windows inside a group do not renormalise; each
// workgroup sums the squared norm after every window, and the finishing
// kernel chains p_g = n_g / (2 n_{g-1}) (n_0 = 1: the first window of the
// group applies sigma) and sets sigma = 1 / sqrt(n_last).
#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kTT = 256;  // threads per workgroup

__device__ __forceinline__ uint32_t ins0u(uint32_t x, int b) { return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1)); }
__device__ __forceinline__ int par64(uint64_t x) { return __popcll(x) & 1; }
__device__ __forceinline__ int par32(uint32_t x) { return __popc(x) & 1; }

// Global index of local element e of the tile whose outer bits are `base`.
__device__ __forceinline__ uint64_t gidx(uint32_t e, uint64_t base, const TileArgs &ta) {
  uint64_t g = base | (e & ((1u << kLowBits) - 1));
  for (int i = kLowBits; i < ta.k; ++i) g |= uint64_t((e >> i) & 1u) << ta.tpos[i];
  return g;
}

// kTB = tile bits (ta.k).  Each thread moves kPer = 2^kTB / kTT amplitudes
// per tile; all its loads are issued before the first LDS store (and all LDS
// reads before the first global store), so the memory system sees kPer
// requests in flight per thread.
template <int kTB>
__global__ __launch_bounds__(kTT) void k_tile(float2 *__restrict__ psi, TileArgs ta, const FuseOp *__restrict__ ops,
                                               MeasureArgs ma, double *__restrict__ partials) {
  constexpr uint32_t kSize = 1u << kTB, kHalf = kSize >> 1;
  constexpr int kPer = kSize / kTT;
  extern __shared__ float2 tile[];
  __shared__ double wacc[kMaxGroupWindows][kTT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool reduce = ma.reduce != kReduceNone;
  if (reduce)
    for (int i = threadIdx.x; i < ta.nwin * (kTT / 64); i += kTT) wacc[i / (kTT / 64)][i % (kTT / 64)] = 0.0;
  const double sg = (ma.reduce == kReduceRenorm) ? *ma.book.sigma : 1.0;
  // the part of each element's global index that comes from threadIdx.x
  const uint64_t g_tid = gidx(threadIdx.x, 0, ta);
  uint64_t g_r[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) g_r[r] = gidx(uint32_t(r) * kTT, 0, ta);
  const uint64_t ntiles = uint64_t(1) << (ta.n - kTB);
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint64_t base = 0;
    for (int i = 0; i < ta.n - kTB; ++i) base |= ((t >> i) & 1) << ta.opos[i];
    float2 v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) v[r] = psi[base | g_tid | g_r[r]];
#pragma unroll
    for (int r = 0; r < kPer; ++r) tile[threadIdx.x + r * kTT] = v[r];
    __syncthreads();
    for (int o = 0; o < ta.nops; ++o) {
      const FuseOp op = ops[o];
      if (op.kind == DK_E || op.kind == DK_Z) {
        if ((base & op.omask_b) == op.omask_b) {
#pragma unroll
          for (int r = 0; r < kPer; ++r) {
            const uint32_t e = threadIdx.x + r * kTT;
            if ((e & op.lmask_b) == op.lmask_b) tile[e] = make_float2(-tile[e].x, -tile[e].y);
          }
        }
      } else if (op.kind == DK_X) {
        const int lb = op.lb;
#pragma unroll
        for (int r = 0; r < kPer / 2; ++r) {
          const uint32_t q = threadIdx.x + r * kTT;
          const uint32_t e0 = ins0u(q, lb), e1 = e0 | (1u << lb);
          const float2 a = tile[e0];
          tile[e0] = tile[e1];
          tile[e1] = a;
        }
      } else {  // window
        const int lb = op.lb;
        const float f = float((op.flags & 16u) ? sg * op.f : double(op.f));
        const float s1 = (op.flags & 8u) ? 1.f : -1.f;
        const int ob = par64(base & op.omask_b), oo = par64(base & op.omask_o1);
        // fold the corrections and the tile-constant signs into the two
        // output coefficients: o0 = f0 (a + c0 b), o1 = f1 (a + c1 b)
        const float2 c = op.coef;
        const bool sw = op.flags & 1u;
        float f0 = f, f1 = (oo ? -f : f);
        float2 c0 = ob ? make_float2(-c.x, -c.y) : c, c1 = make_float2(s1 * c0.x, s1 * c0.y);
        if (op.flags & 2u) { if (sw) f1 = -f1; else f0 = -f0; }
        if (op.flags & 4u) { if (sw) f0 = -f0; else f1 = -f1; }
        float acc = 0.f;  // per-thread partial of at most kPer/2 pairs; FP64 from the wave sum on
        if (op.lmask_b == 0 && op.lmask_o1 == 0) {
#pragma unroll
          for (int r = 0; r < kPer / 2; ++r) {
            const uint32_t q = threadIdx.x + r * kTT;
            const uint32_t e0 = ins0u(q, lb), e1 = e0 | (1u << lb);
            const float2 a = tile[e0], b = tile[e1];
            const float2 p0 = make_float2(f0 * (a.x + (c0.x * b.x - c0.y * b.y)), f0 * (a.y + (c0.x * b.y + c0.y * b.x)));
            const float2 p1 = make_float2(f1 * (a.x + (c1.x * b.x - c1.y * b.y)), f1 * (a.y + (c1.x * b.y + c1.y * b.x)));
            tile[e0] = sw ? p1 : p0;
            tile[e1] = sw ? p0 : p1;
            acc += p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y;
          }
        } else {
#pragma unroll
          for (int r = 0; r < kPer / 2; ++r) {
            const uint32_t q = threadIdx.x + r * kTT;
            const uint32_t e0 = ins0u(q, lb), e1 = e0 | (1u << lb);
            const float sb = par32(e0 & op.lmask_b) ? -1.f : 1.f;
            const float so1 = par32(e0 & op.lmask_o1) ? -1.f : 1.f;
            const float2 a = tile[e0], b0 = tile[e1];
            const float2 b = make_float2(sb * b0.x, sb * b0.y);
            const float g1 = so1 * f1;
            const float2 p0 = make_float2(f0 * (a.x + (c0.x * b.x - c0.y * b.y)), f0 * (a.y + (c0.x * b.y + c0.y * b.x)));
            const float2 p1 = make_float2(g1 * (a.x + (c1.x * b.x - c1.y * b.y)), g1 * (a.y + (c1.x * b.y + c1.y * b.x)));
            tile[e0] = sw ? p1 : p0;
            tile[e1] = sw ? p0 : p1;
            acc += p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y;
          }
        }
        if (reduce) {
          double d = acc;
          for (int off = 32; off > 0; off >>= 1) d += __shfl_down(d, off, 64);
          if (lane == 0) wacc[op.widx][wave] += d;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) v[r] = tile[threadIdx.x + r * kTT];
#pragma unroll
    for (int r = 0; r < kPer; ++r) psi[base | g_tid | g_r[r]] = v[r];
    __syncthreads();
  }
  if (reduce) {
    for (int w = threadIdx.x; w < ta.nwin; w += kTT) {
      double s = 0.0;
      for (int k = 0; k < kTT / 64; ++k) s += wacc[w][k];
      partials[size_t(w) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Group finish, one workgroup per window g of the group (all in parallel):
// block g sums the partials of windows g-1 and g in block order, records
// p_g = n_g / (2 n_{g-1}) (n_{-1} = 1: the first window applies sigma) and
// checks it; the block of the last window sets sigma = 1 / sqrt(n_last).
__device__ double sum_partials(const double *part, unsigned nblk) {
  __shared__ double red[kTT / 64];
  constexpr int kLoads = kTileGridCap / kTT;  // nblk <= kTileGridCap
  double v[kLoads];
#pragma unroll
  for (int k = 0; k < kLoads; ++k) {
    const unsigned i = threadIdx.x + unsigned(k) * kTT;
    v[k] = i < nblk ? part[i] : 0.0;
  }
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kLoads; ++k) t += v[k];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = t;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kTT / 64; ++k) s += red[k];
  return s;
}

__global__ __launch_bounds__(kTT) void k_finish_group(DevBook book, const int *__restrict__ m_of_window, int nwin,
                                                       unsigned nblk, int reduce) {
  const int g = blockIdx.x;
  const double n = sum_partials(book.partials + size_t(g) * nblk, nblk);
  const double prev = g > 0 ? sum_partials(book.partials + size_t(g - 1) * nblk, nblk) : 1.0;
  if (threadIdx.x != 0) return;
  const double p = prev > 0.0 ? 0.5 * n / prev : 0.0;
  const int m = m_of_window[g];
  book.probs[m] = p;
  if (reduce == kReduceRenorm && p < 1e-10) {
    atomicMin(&book.err[0], m);
    book.err[1] = kErrZeroProb;
  } else if (reduce == kReduceCheck && fabs(p - 0.5) > 1e-4) {
    atomicMin(&book.err[0], m);
    book.err[1] = kErrNotDet;
  }
  if (reduce == kReduceRenorm && g == nwin - 1) *book.sigma = n > 1e-300 ? 1.0 / sqrt(n) : 0.0;
}

}  // namespace

unsigned tile_grid(const TileArgs &ta) {
  const uint64_t ntiles = uint64_t(1) << (ta.n - ta.k);
  return unsigned(ntiles < kTileGridCap ? ntiles : kTileGridCap);
}

hipError_t tile_prepare() {
  hipError_t e = hipSuccess;
  const void *fns[] = {reinterpret_cast<const void *>(k_tile<10>), reinterpret_cast<const void *>(k_tile<11>),
                       reinterpret_cast<const void *>(k_tile<12>), reinterpret_cast<const void *>(k_tile<13>)};
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, int(sizeof(float2) << (10 + i)));
  return e;
}

hipError_t launch_tile(float2 *psi, const TileArgs &ta, const FuseOp *ops, const MeasureArgs &a, hipStream_t s,
                       unsigned *grid) {
  const size_t bytes = sizeof(float2) << ta.k;
  const unsigned g = tile_grid(ta);
  switch (ta.k) {
    case 10: hipLaunchKernelGGL(k_tile<10>, dim3(g), dim3(kTT), bytes, s, psi, ta, ops, a, a.book.partials); break;
    case 11: hipLaunchKernelGGL(k_tile<11>, dim3(g), dim3(kTT), bytes, s, psi, ta, ops, a, a.book.partials); break;
    case 12: hipLaunchKernelGGL(k_tile<12>, dim3(g), dim3(kTT), bytes, s, psi, ta, ops, a, a.book.partials); break;
    case 13: hipLaunchKernelGGL(k_tile<13>, dim3(g), dim3(kTT), bytes, s, psi, ta, ops, a, a.book.partials); break;
    default: return hipErrorInvalidValue;
  }
  *grid = g;
  return hipGetLastError();
}

hipError_t launch_finish_group(const MeasureArgs &a, const int *m_of_window, int nwin, unsigned nblk,
                               hipStream_t s) {
  // a group without windows changes no norm: sigma stays as it is
  if (a.reduce == kReduceNone || nwin == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_finish_group, dim3(nwin), dim3(kTT), 0, s, a.book, m_of_window, nwin, nblk, a.reduce);
  return hipGetLastError();
}

}  // namespace owqs
