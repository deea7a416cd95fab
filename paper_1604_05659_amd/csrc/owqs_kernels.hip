// owqs_kernels.hip -- gfx950 kernels for 1WQC pattern execution.
//
// The live state is one complex64 vector (float2, interleaved re/im) of 2^n
// amplitudes; bit k of an index is the qubit the host's slot map assigns to
// slot k.  Every kernel streams HBM with 16-byte accesses (float4 = two
// amplitudes) through grid-stride loops; no kernel uses MFMA because none of
// these commands is a dense contraction.
//
// Commands and the paper's passages they implement:
//   prepare  (N,   Sec. 2.2 / 4.4.1): psi (x) |+>; the new qubit takes the top
//            slot n, so the vector doubles by copying the lower half up (the
//            1/sqrt 2 is kept on the host and folded into the next M).
//   cz       (E,   Sec. 4.4.1, Fig. 5): negate the quarter with both bits 1.
//   pauli_x/z(X/Z, Sec. 4.4.1): swap pairs / negate the bit-b = 1 half.
//   measure  (M,   Sec. 4.2, 4.4.2, Eqs. 11-13, Fig. 6): forced-outcome
//            elimination out = f (psi0 + c psi1), with the FP64 outcome
//            probability reduced in the same pass.  In place: the vector
//            halves by moving the top qubit into the measured slot, so the
//            pass reads every amplitude once and writes half of them.
//   jwindow  (N w; E's on v or w; M v; X/Z on w): the same window done as
//            one 2x2 update of slot(v) in place (the new qubit w takes v's
//            slot); E's touching other qubits become index-parity signs.
//   read     : gather the outputs into the caller's bit order, scaled by the
//            FP64 factor.
#include <climits>

#include "owqs_gather.h"
#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kBlock = 256;   // 4 wave64 per block
constexpr int kUnroll = 2;    // 16-byte units per thread per loop trip
constexpr unsigned kGridCap = 4096;

__device__ __forceinline__ uint64_t ins0(uint64_t x, int b) {
  const uint64_t lo = x & ((uint64_t(1) << b) - 1);
  return ((x >> b) << (b + 1)) | lo;
}
__device__ __forceinline__ uint64_t ins1(uint64_t x, int b) { return ins0(x, b) | (uint64_t(1) << b); }

__device__ __forceinline__ float4 ld4(const float2 *p, uint64_t i) {
  return *reinterpret_cast<const float4 *>(p + i);
}
__device__ __forceinline__ void st4(float2 *p, uint64_t i, float4 v) {
  *reinterpret_cast<float4 *>(p + i) = v;
}

// Streaming forms with the non-temporal hint (loads and stores).  Measured on
// MI355X: above the 256 MB Infinity Cache (live width >= 26) they lift N and
// M from about 0.60 to 0.70 of HBM peak; at 2^24 and 2^25, where the next
// kernel re-reads the vector from that cache, the plain forms are faster.
typedef float f4v __attribute__((ext_vector_type(4)));
template <bool kNT>
__device__ __forceinline__ float4 ldv(const float2 *p, uint64_t i) {
  if (kNT) {
    const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p + i));
    return make_float4(x.x, x.y, x.z, x.w);
  }
  return ld4(p, i);
}
template <bool kNT>
__device__ __forceinline__ void stv(float2 *p, uint64_t i, float4 v) {
  if (kNT) {
    const f4v x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<f4v *>(p + i));
  } else {
    st4(p, i, v);
  }
}
constexpr int kNtWidthNM = 26;  // M at live width n >= 26, N producing width >= 26
constexpr int kNtWidthX = 26;   // X at live width n >= 26 (at 25 the plain form measured faster)
__device__ __forceinline__ float2 lo2(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 pack(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }

// f * (a + c * b)
__device__ __forceinline__ float2 axpc(float2 a, float2 c, float2 b, float f) {
  const float re = a.x + (c.x * b.x - c.y * b.y);
  const float im = a.y + (c.x * b.y + c.y * b.x);
  return make_float2(f * re, f * im);
}
__device__ __forceinline__ double nrm2(float2 v) {
  return double(v.x) * double(v.x) + double(v.y) * double(v.y);
}

#define GRID_STRIDE_UNITS(units)                                                           \
  for (uint64_t base_ = uint64_t(blockIdx.x) * (kBlock * kUnroll) + threadIdx.x; base_ < (units); \
       base_ += uint64_t(gridDim.x) * (kBlock * kUnroll))

unsigned grid_for(uint64_t units) {
  const uint64_t per = uint64_t(kBlock) * kUnroll;
  uint64_t g = (units + per - 1) / per;
  if (g < 1) g = 1;
  if (g > kGridCap) g = kGridCap;
  return unsigned(g);
}

// ---------------------------------------------------------------------------
// FP64 reduction, stage 1: every block writes the sum of |out|^2 over its
// threads to partials[blockIdx.x] (fixed order inside the block).  Stage 2 is
// k_finish_measure, launched right after on the same stream, so the kernel
// boundary orders the partial stores before their reads (no device-scope
// fences inside the streaming kernel).
// ---------------------------------------------------------------------------
__device__ void block_partial(double acc, double *partials) {
  __shared__ double wsum[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += wsum[w];
    partials[blockIdx.x] = s;
  }
}

// Stage 2 (one block): sum the partials in block order, record p = sum / 2
// for measurement m and, in OWQS mode, set sigma = 1 / sqrt(sum).
__global__ __launch_bounds__(kBlock) void k_finish_measure(DevBook book, unsigned nparts, int m_index,
                                                            int reduce) {
  __shared__ double wsum[kBlock / 64];
  // nparts <= kGridCap = 16 * kBlock: issue all loads before summing
  constexpr int kPer = kGridCap / kBlock;
  double v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const unsigned i = threadIdx.x + unsigned(k) * kBlock;
    v[k] = i < nparts ? book.partials[i] : 0.0;
  }
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) t += v[k];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) sum += wsum[w];
    const double p = 0.5 * sum;
    book.probs[m_index] = p;
    if (reduce == kReduceRenorm) {
      if (p < 1e-10) {
        atomicMin(&book.err[0], m_index);
        book.err[1] = kErrZeroProb;
        *book.sigma = 0.0;
      } else {
        *book.sigma = 1.0 / sqrt(sum);
      }
    } else if (reduce == kReduceCheck) {
      if (fabs(p - 0.5) > 1e-4) {
        atomicMin(&book.err[0], m_index);
        book.err[1] = kErrNotDet;
      }
    }
  }
}

__device__ __forceinline__ float scale_of(const MeasureArgs &a) {
  const double sg = (a.reduce == kReduceRenorm) ? *a.book.sigma : 1.0;
  return float(sg * a.host_factor);
}

// ---------------------------------------------------------------------------
__global__ void k_init(float2 *psi, DevBook book, int set_one) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (set_one) psi[0] = make_float2(1.f, 0.f);
    *book.sigma = 1.0;
    book.err[0] = kErrNone;
    book.err[1] = 0;
  }
}

// N: psi[i + 2^n] = psi[i]; units of two amplitudes (n >= 1).
template <bool kNT>
__global__ __launch_bounds__(kBlock) void k_prepare(float2 *__restrict__ psi, uint64_t units, uint64_t dim) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) v[k] = ldv<kNT>(psi, 2 * u);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) stv<kNT>(psi, 2 * u + dim, v[k]);
    }
  }
}

__global__ void k_prepare_scalar(float2 *psi) { psi[1] = psi[0]; }  // n = 0

// E with both bits >= 1: negate whole 16-byte units of the |11> quarter.
__global__ __launch_bounds__(kBlock) void k_cz_v(float2 *__restrict__ psi, uint64_t units, int lo, int hi) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
    uint64_t j[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      j[k] = ins1(ins1(2 * u, lo), hi);
      if (u < units) v[k] = ld4(psi, j[k]);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) st4(psi, j[k], make_float4(-v[k].x, -v[k].y, -v[k].z, -v[k].w));
    }
  }
}

// E with one bit = 0: the odd amplitude of every unit in the bit-hi = 1 half.
__global__ __launch_bounds__(kBlock) void k_cz_b0(float2 *__restrict__ psi, uint64_t units, int hi) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
    uint64_t j[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      j[k] = ins1(2 * u, hi);
      if (u < units) v[k] = ld4(psi, j[k]);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) st4(psi, j[k], make_float4(v[k].x, v[k].y, -v[k].z, -v[k].w));
    }
  }
}

// X on bit b >= 1: swap unit j with unit j + 2^b.
template <bool kNT>
__global__ __launch_bounds__(kBlock) void k_x_v(float2 *__restrict__ psi, uint64_t units, int b) {
  const uint64_t step = uint64_t(1) << b;
  GRID_STRIDE_UNITS(units) {
    float4 x[kUnroll], y[kUnroll];
    uint64_t j[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      j[k] = ins0(2 * u, b);
      if (u < units) {
        x[k] = ldv<kNT>(psi, j[k]);
        y[k] = ldv<kNT>(psi, j[k] + step);
      }
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) {
        stv<kNT>(psi, j[k], y[k]);
        stv<kNT>(psi, j[k] + step, x[k]);
      }
    }
  }
}

// X on bit 0: swap the two amplitudes inside every unit.
template <bool kNT>
__global__ __launch_bounds__(kBlock) void k_x_b0(float2 *__restrict__ psi, uint64_t units) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) v[k] = ldv<kNT>(psi, 2 * u);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) stv<kNT>(psi, 2 * u, make_float4(v[k].z, v[k].w, v[k].x, v[k].y));
    }
  }
}

// Z on bit b >= 1: negate the units of the bit-b = 1 half.
__global__ __launch_bounds__(kBlock) void k_z_v(float2 *__restrict__ psi, uint64_t units, int b) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
    uint64_t j[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      j[k] = ins1(2 * u, b);
      if (u < units) v[k] = ld4(psi, j[k]);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) st4(psi, j[k], make_float4(-v[k].x, -v[k].y, -v[k].z, -v[k].w));
    }
  }
}

// Z on bit 0: negate the odd amplitude of every unit.
__global__ __launch_bounds__(kBlock) void k_z_b0(float2 *__restrict__ psi, uint64_t units) {
  GRID_STRIDE_UNITS(units) {
    float4 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) v[k] = ld4(psi, 2 * u);
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const uint64_t u = base_ + uint64_t(k) * kBlock;
      if (u < units) st4(psi, 2 * u, make_float4(v[k].x, v[k].y, -v[k].z, -v[k].w));
    }
  }
}

// Scalar forms for live widths below 3 (a handful of amplitudes; one thread).
__global__ void k_small_cmd(float2 *psi, int n, int op, int b0, int b1) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t dim = uint64_t(1) << n;
  for (uint64_t i = 0; i < dim; ++i) {
    if (op == 1) {  // E
      if (((i >> b0) & 1) && ((i >> b1) & 1)) psi[i] = make_float2(-psi[i].x, -psi[i].y);
    } else if (op == 3) {  // X
      if (!((i >> b0) & 1)) {
        const float2 t = psi[i];
        psi[i] = psi[i | (uint64_t(1) << b0)];
        psi[i | (uint64_t(1) << b0)] = t;
      }
    } else if (op == 4) {  // Z
      if ((i >> b0) & 1) psi[i] = make_float2(-psi[i].x, -psi[i].y);
    }
  }
}

// ---------------------------------------------------------------------------
// M, move-to-top layout.  t = n - 1, H = 2^t.  For every index j < H with
// bit b = 0 (b < t):
//   out[j]       = f (psi[j]     + c psi[j + 2^b])      (top qubit = 0)
//   out[j + 2^b] = f (psi[j + H] + c psi[j + 2^b + H])  (top qubit = 1)
// so afterwards slot b holds the former top qubit.  For b = t:
//   out[j] = f (psi[j] + c psi[j + H]).
// Each thread reads only the four (two) amplitudes it writes, so the update
// is race-free in place.
// ---------------------------------------------------------------------------
template <int kCase, bool kNT>  // kCase 0: b == t, 1: b == 0 < t, 2: 1 <= b < t
__global__ __launch_bounds__(kBlock) void k_measure(float2 *__restrict__ psi, uint64_t units, int b,
                                                     uint64_t half, MeasureArgs a) {
  const float f = scale_of(a);
  const float2 c = a.coef_dev ? *a.coef_dev : a.coef;
  const uint64_t step = uint64_t(1) << b;
  double acc = 0.0;
  GRID_STRIDE_UNITS(units) {
    if (kCase == 2) {
      float4 A[kUnroll], B[kUnroll], C[kUnroll], D[kUnroll];
      uint64_t j[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        j[k] = ins0(2 * u, b);
        if (u < units) {
          A[k] = ldv<kNT>(psi, j[k]);
          B[k] = ldv<kNT>(psi, j[k] + step);
          C[k] = ldv<kNT>(psi, j[k] + half);
          D[k] = ldv<kNT>(psi, j[k] + step + half);
        }
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) {
          const float2 o0 = axpc(lo2(A[k]), c, lo2(B[k]), f);
          const float2 o1 = axpc(hi2(A[k]), c, hi2(B[k]), f);
          const float2 o2 = axpc(lo2(C[k]), c, lo2(D[k]), f);
          const float2 o3 = axpc(hi2(C[k]), c, hi2(D[k]), f);
          stv<kNT>(psi, j[k], pack(o0, o1));
          stv<kNT>(psi, j[k] + step, pack(o2, o3));
          acc += nrm2(o0) + nrm2(o1) + nrm2(o2) + nrm2(o3);
        }
      }
    } else {
      float4 X[kUnroll], Y[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) {
          X[k] = ldv<kNT>(psi, 2 * u);
          Y[k] = ldv<kNT>(psi, 2 * u + half);
        }
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) {
          float2 o0, o1;
          if (kCase == 0) {
            o0 = axpc(lo2(X[k]), c, lo2(Y[k]), f);
            o1 = axpc(hi2(X[k]), c, hi2(Y[k]), f);
          } else {
            o0 = axpc(lo2(X[k]), c, hi2(X[k]), f);
            o1 = axpc(lo2(Y[k]), c, hi2(Y[k]), f);
          }
          stv<kNT>(psi, 2 * u, pack(o0, o1));
          acc += nrm2(o0) + nrm2(o1);
        }
      }
    }
  }
  if (a.reduce != kReduceNone) block_partial(acc, a.book.partials);
}

// M at live widths 1 and 2 (one thread; same move-to-top layout).
__global__ void k_measure_small(float2 *psi, int n, int b, MeasureArgs a) {
  double acc = 0.0;
  if (threadIdx.x == 0) {
    const float f = scale_of(a);
    const int t = n - 1;
    const uint64_t half = uint64_t(1) << t;
    float2 in[4];
    for (uint64_t i = 0; i < (uint64_t(1) << n); ++i) in[i] = psi[i];
    float2 out[2];
    for (uint64_t j = 0; j < half; ++j) {
      uint64_t k0;
      if (b == t || !((j >> b) & 1)) {
        k0 = j;
      } else {
        k0 = (j & ~(uint64_t(1) << b)) + half;
      }
      out[j] = axpc(in[k0], a.coef_dev ? *a.coef_dev : a.coef, in[k0 | (uint64_t(1) << b)], f);
    }
    for (uint64_t j = 0; j < half; ++j) {
      psi[j] = out[j];
      acc += nrm2(out[j]);
    }
  }
  if (a.reduce != kReduceNone) block_partial(acc, a.book.partials);
}

// ---------------------------------------------------------------------------
// Window N w; E...; M v; (X|Z on w)*: one in-place 2x2 pass over v's slot b
// (see Window): o0 = f (a + c sb b), o1 = so1 f (a + s c sb b), then the
// folded corrections; w takes slot b.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sgn_of(uint64_t j, uint64_t mask) {
  return (__popcll(j & mask) & 1) ? -1.f : 1.f;
}

__device__ __forceinline__ void window_pair(float2 a, float2 bb, uint64_t j, float2 c, float f, const Window &w,
                                            float2 &o0, float2 &o1) {
  const float sb = sgn_of(j, w.mask_b), so1 = sgn_of(j, w.mask_o1);
  float2 cb = make_float2(sb * (c.x * bb.x - c.y * bb.y), sb * (c.x * bb.y + c.y * bb.x));
  o0 = make_float2(f * (a.x + cb.x), f * (a.y + cb.y));
  const float s = w.vw_even ? 1.f : -1.f;
  o1 = make_float2(so1 * f * (a.x + s * cb.x), so1 * f * (a.y + s * cb.y));
  if (w.swap) { const float2 t = o0; o0 = o1; o1 = t; }
  if (w.neg0) o0 = make_float2(-o0.x, -o0.y);
  if (w.neg1) o1 = make_float2(-o1.x, -o1.y);
}

template <bool kB0>
__global__ __launch_bounds__(kBlock) void k_jwindow(float2 *__restrict__ psi, uint64_t units, int b,
                                                     MeasureArgs a, Window win) {
  const float f = scale_of(a);
  const float2 c = a.coef_dev ? *a.coef_dev : a.coef;
  if (a.fold_dev) {  // corrections resolved on the device (drawn outcomes)
    win.swap = a.fold_dev[0];
    win.neg0 = a.fold_dev[1];
    win.neg1 = a.fold_dev[2];
  }
  const uint64_t step = uint64_t(1) << b;
  double acc = 0.0;
  GRID_STRIDE_UNITS(units) {
    if (!kB0) {
      float4 A[kUnroll], B[kUnroll];
      uint64_t j[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        j[k] = ins0(2 * u, b);
        if (u < units) {
          A[k] = ld4(psi, j[k]);
          B[k] = ld4(psi, j[k] + step);
        }
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) {
          float2 p0, q0, p1, q1;
          window_pair(lo2(A[k]), lo2(B[k]), j[k], c, f, win, p0, q0);
          window_pair(hi2(A[k]), hi2(B[k]), j[k] + 1, c, f, win, p1, q1);
          st4(psi, j[k], pack(p0, p1));
          st4(psi, j[k] + step, pack(q0, q1));
          acc += nrm2(p0) + nrm2(p1) + nrm2(q0) + nrm2(q1);
        }
      }
    } else {
      float4 X[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) X[k] = ld4(psi, 2 * u);
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const uint64_t u = base_ + uint64_t(k) * kBlock;
        if (u < units) {
          float2 p, q;
          window_pair(lo2(X[k]), hi2(X[k]), 2 * u, c, f, win, p, q);
          st4(psi, 2 * u, pack(p, q));
          acc += nrm2(p) + nrm2(q);
        }
      }
    }
  }
  if (a.reduce != kReduceNone) block_partial(acc, a.book.partials);
  if (a.prob_half && blockIdx.x == 0 && threadIdx.x == 0) a.book.probs[a.m_index] = 0.5;
}

// ---------------------------------------------------------------------------
struct Where {
  int bit[kWhereMax];
};

__global__ __launch_bounds__(kGatherThreads) void k_read(const float2 *__restrict__ psi, float2 *__restrict__ out,
                                                          int nout, Where w, double host_factor, const double *sigma) {
  __shared__ uint64_t tab[1 << kGatherLo];
  const double sg = sigma ? *sigma : 1.0;
  gather_chunks(psi, out, nout, w.bit, float(sg * host_factor), tab, blockIdx.x, gridDim.x);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(float2 *psi, DevBook book, hipStream_t s, int set_one) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, psi, book, set_one);
  return hipGetLastError();
}

hipError_t launch_prepare(float2 *psi, int n, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(k_prepare_scalar, dim3(1), dim3(1), 0, s, psi);
  } else {
    const uint64_t units = uint64_t(1) << (n - 1);
    if (n + 1 >= kNtWidthNM)
      hipLaunchKernelGGL(k_prepare<true>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, uint64_t(1) << n);
    else
      hipLaunchKernelGGL(k_prepare<false>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, uint64_t(1) << n);
  }
  return hipGetLastError();
}

hipError_t launch_cz(float2 *psi, int n, int b0, int b1, hipStream_t s) {
  const int lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
  if (n < 3) {
    hipLaunchKernelGGL(k_small_cmd, dim3(1), dim3(64), 0, s, psi, n, 1, lo, hi);
  } else if (lo >= 1) {
    const uint64_t units = uint64_t(1) << (n - 3);
    hipLaunchKernelGGL(k_cz_v, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, lo, hi);
  } else {
    const uint64_t units = uint64_t(1) << (n - 2);
    hipLaunchKernelGGL(k_cz_b0, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, hi);
  }
  return hipGetLastError();
}

hipError_t launch_pauli_x(float2 *psi, int n, int b, hipStream_t s) {
  if (n < 3) {
    hipLaunchKernelGGL(k_small_cmd, dim3(1), dim3(64), 0, s, psi, n, 3, b, 0);
  } else if (b >= 1) {
    const uint64_t units = uint64_t(1) << (n - 2);
    if (n >= kNtWidthX)
      hipLaunchKernelGGL(k_x_v<true>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, b);
    else
      hipLaunchKernelGGL(k_x_v<false>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, b);
  } else {
    const uint64_t units = uint64_t(1) << (n - 1);
    if (n >= kNtWidthX)
      hipLaunchKernelGGL(k_x_b0<true>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units);
    else
      hipLaunchKernelGGL(k_x_b0<false>, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units);
  }
  return hipGetLastError();
}

hipError_t launch_pauli_z(float2 *psi, int n, int b, hipStream_t s) {
  if (n < 3) {
    hipLaunchKernelGGL(k_small_cmd, dim3(1), dim3(64), 0, s, psi, n, 4, b, 0);
  } else if (b >= 1) {
    const uint64_t units = uint64_t(1) << (n - 2);
    hipLaunchKernelGGL(k_z_v, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units, b);
  } else {
    const uint64_t units = uint64_t(1) << (n - 1);
    hipLaunchKernelGGL(k_z_b0, dim3(grid_for(units)), dim3(kBlock), 0, s, psi, units);
  }
  return hipGetLastError();
}

hipError_t launch_finish(const MeasureArgs &a, unsigned nparts, hipStream_t s) {
  if (a.reduce == kReduceNone) return hipGetLastError();
  hipLaunchKernelGGL(k_finish_measure, dim3(1), dim3(kBlock), 0, s, a.book, nparts, a.m_index, a.reduce);
  return hipGetLastError();
}

hipError_t launch_measure(float2 *psi, int n, int b, const MeasureArgs &a, hipStream_t s, unsigned *grid) {
  const int t = n - 1;
  const uint64_t half = uint64_t(1) << t;
  unsigned g = 1;
  if (n < 3) {
    hipLaunchKernelGGL(k_measure_small, dim3(1), dim3(kBlock), 0, s, psi, n, b, a);
  } else if (b == t) {
    const uint64_t units = uint64_t(1) << (n - 2);
    g = grid_for(units);
    if (n >= kNtWidthNM)
      hipLaunchKernelGGL((k_measure<0, true>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
    else
      hipLaunchKernelGGL((k_measure<0, false>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
  } else if (b == 0) {
    const uint64_t units = uint64_t(1) << (n - 2);
    g = grid_for(units);
    if (n >= kNtWidthNM)
      hipLaunchKernelGGL((k_measure<1, true>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
    else
      hipLaunchKernelGGL((k_measure<1, false>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
  } else {
    const uint64_t units = uint64_t(1) << (n - 3);
    g = grid_for(units);
    if (n >= kNtWidthNM)
      hipLaunchKernelGGL((k_measure<2, true>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
    else
      hipLaunchKernelGGL((k_measure<2, false>), dim3(g), dim3(kBlock), 0, s, psi, units, b, half, a);
  }
  *grid = g;
  return hipGetLastError();
}

hipError_t launch_jwindow(float2 *psi, int n, int b, const MeasureArgs &a, const Window &win, hipStream_t s,
                          unsigned *grid) {
  unsigned g;
  if (b >= 1) {
    const uint64_t units = uint64_t(1) << (n - 2);
    g = grid_for(units);
    hipLaunchKernelGGL(k_jwindow<false>, dim3(g), dim3(kBlock), 0, s, psi, units, b, a, win);
  } else {
    const uint64_t units = uint64_t(1) << (n - 1);
    g = grid_for(units);
    hipLaunchKernelGGL(k_jwindow<true>, dim3(g), dim3(kBlock), 0, s, psi, units, b, a, win);
  }
  *grid = g;
  return hipGetLastError();
}

hipError_t launch_read(const float2 *psi, float2 *out, int nout, const int *where, double host_factor,
                       const double *sigma, hipStream_t s) {
  Where w{};
  for (int k = 0; k < nout; ++k) w.bit[k] = where[k];
  // one chunk of 2^kGatherLo outputs per workgroup and trip
  const int lo = nout < kGatherLo ? nout : kGatherLo;
  uint64_t g = uint64_t(1) << (nout - lo);
  if (g > kGridCap) g = kGridCap;
  hipLaunchKernelGGL(k_read, dim3(unsigned(g)), dim3(kGatherThreads), 0, s, psi, out, nout, w, host_factor, sigma);
  return hipGetLastError();
}

}  // namespace owqs
