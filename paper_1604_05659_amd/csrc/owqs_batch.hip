// owqs_batch.hip -- whole patterns resident in LDS (live width <= 14).
//
// One workgroup runs one pattern instance from its first command to the
// read-out without touching HBM in between: the live vector (2^n complex64,
// at most 128 KiB) sits in the 160 KiB LDS of a gfx950 CU, every command is a
// strided pass over it separated by workgroup barriers, and the FP64
// probability reduction of an M (Eq. 13) is a workgroup reduction, so the
// renormalisation scale (Eq. 7) never leaves the CU.  HBM traffic is the
// command table, the input and the output only.
//
// Used for batches of many small patterns (each item its own command table)
// and for the recognition problem (one table, every computational-basis
// input: column k of the unitary is the output for |k>).
#include <algorithm>

#include "owqs_gather.h"
#include "owqs_internal.h"

namespace owqs {
namespace {

// Workgroup size by live width: one wave64 up to width 8 (its barriers are
// nearly free), 4 waves up to width 11, 8 waves above.
constexpr int threads_for(int width) { return width <= 8 ? 64 : width <= 11 ? 256 : 512; }

__device__ __forceinline__ uint32_t i0(uint32_t x, int b) { return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1)); }

__device__ __forceinline__ float2 fma_c(float2 a, float2 c, float2 b, float f, float sgn) {
  const float re = a.x + sgn * (c.x * b.x - c.y * b.y);
  const float im = a.y + sgn * (c.x * b.y + c.y * b.x);
  return make_float2(f * re, f * im);
}
__device__ __forceinline__ double n2(float2 v) { return double(v.x) * v.x + double(v.y) * v.y; }
__device__ __forceinline__ float2 neg(float2 v) { return make_float2(-v.x, -v.y); }

// Sum of v over the workgroup, the same value returned to every thread.
template <int kT>
__device__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kT / 64; ++k) s += red[k];
  return s;
}

// One command row, read as whole dwords through the constant address space
// (the table is never written by the kernels), so the scalar unit loads it:
// every thread of the workgroup walks the same command list.
__device__ __forceinline__ DevStep load_step(const DevStep *steps, int s) {
  static_assert(sizeof(DevStep) % 4 == 0, "DevStep is whole dwords");
  constexpr int kWords = sizeof(DevStep) / 4;
  typedef const __attribute__((address_space(4))) uint32_t cword;
  cword *src = reinterpret_cast<cword *>(reinterpret_cast<uintptr_t>(steps)) + kWords * __builtin_amdgcn_readfirstlane(s);
  uint32_t w[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = src[i];
  DevStep st;
  __builtin_memcpy(&st, w, sizeof(st));
  return st;
}

template <int kT>
__device__ void run_item(const DevStep *__restrict__ steps, int nsteps, int nin, int nout, const int *where,
                         double final_factor, float2 *lds, const float2 *__restrict__ in, int basis,
                         float2 *__restrict__ out, double *__restrict__ probs, int reduce, int *err, int item,
                         double *red) {
  // item < 0: report the failing measurement index instead of the item.
  // Input: |basis> when basis >= 0, else in[0 .. 2^nin); a pattern without
  // inputs (nin = 0) and no input pointer starts from the empty product
  // state (the single amplitude 1).  The host never passes in == nullptr
  // with nin > 0.
  const uint32_t din = 1u << nin;
  for (uint32_t i = threadIdx.x; i < din; i += kT) {
    float2 v;
    if (basis >= 0) v = make_float2(i == uint32_t(basis) ? 1.f : 0.f, 0.f);
    else if (in) v = in[i];
    else v = make_float2(i == 0 ? 1.f : 0.f, 0.f);
    lds[i] = v;
  }
  double sigma = 1.0;
  int half_run = 0;  // windows in a row recorded with p = 1/2 and no sum (at most kHalfRun)
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    const DevStep st = load_step(steps, s);
    const uint32_t dim = 1u << st.n;
    const int b = st.b0;
    if (st.kind == DK_N) {
      for (uint32_t i = threadIdx.x; i < dim; i += kT) lds[i + dim] = lds[i];
    } else if (st.kind == DK_E) {
      const int lo = st.b0 < st.b1 ? st.b0 : st.b1, hi = st.b0 < st.b1 ? st.b1 : st.b0;
      const uint32_t set = (1u << lo) | (1u << hi);
      for (uint32_t i = threadIdx.x; i < (dim >> 2); i += kT) {
        const uint32_t j = i0(i0(i, lo), hi) | set;
        lds[j] = neg(lds[j]);
      }
    } else if (st.kind == DK_X) {
      for (uint32_t i = threadIdx.x; i < (dim >> 1); i += kT) {
        const uint32_t j = i0(i, b);
        const float2 t = lds[j];
        lds[j] = lds[j + (1u << b)];
        lds[j + (1u << b)] = t;
      }
    } else if (st.kind == DK_Z) {
      for (uint32_t i = threadIdx.x; i < (dim >> 1); i += kT) {
        const uint32_t j = i0(i, b) | (1u << b);
        lds[j] = neg(lds[j]);
      }
    } else if (st.kind == DK_U) {  // windows on slot b composed into one map, none summed
      uint32_t w[6];
      __builtin_memcpy(&w[0], &st.host_factor, 4);
      w[1] = st.pp;
      w[2] = uint32_t(st.mask_b);
      w[3] = uint32_t(st.mask_b >> 32);
      w[4] = uint32_t(st.mask_o1);
      w[5] = uint32_t(st.mask_o1 >> 32);
      float e[6];
      __builtin_memcpy(e, w, sizeof(e));
      const float2 m00 = st.coef, m01 = make_float2(e[0], e[1]), m10 = make_float2(e[2], e[3]),
                   m11 = make_float2(e[4], e[5]);
      for (uint32_t i = threadIdx.x; i < (dim >> 1); i += kT) {
        const uint32_t j = i0(i, b), st2 = 1u << b;
        const float2 a = lds[j], bb = lds[j + st2];
        lds[j] = make_float2(m00.x * a.x - m00.y * a.y + m01.x * bb.x - m01.y * bb.y,
                             m00.x * a.y + m00.y * a.x + m01.x * bb.y + m01.y * bb.x);
        lds[j + st2] = make_float2(m10.x * a.x - m10.y * a.y + m11.x * bb.x - m11.y * bb.y,
                                   m10.x * a.y + m10.y * a.x + m11.x * bb.y + m11.y * bb.x);
      }
      if (reduce == kReduceRenorm) {  // OWQS: each of its b1 windows has p = 1/2 (indices after the rows)
        const int *ml = reinterpret_cast<const int *>(steps + nsteps) + st.m_index;
        if (probs)
          for (int k = threadIdx.x; k < int(st.b1); k += kT) probs[ml[k]] = 0.5;
        half_run += int(st.b1);
      }
    } else {  // DK_M or DK_J
      // OWQS: a window with an odd E(v, w) count has p = 1/2 exactly for every
      // state (Eqs. 11-13): it is recorded without the block sum and sigma is
      // left for the next measurement that sums (at most kHalfRun in a row)
      const bool half = reduce == kReduceRenorm && st.kind == DK_J && !(st.pp & 24u) && half_run < kHalfRun;
      const float f = float((reduce == kReduceRenorm && !half ? sigma : 1.0) * st.host_factor);
      const float2 c = st.coef;
      double acc = 0.0;
      if (st.kind == DK_M) {
        const int t = st.n - 1;
        const uint32_t half = 1u << t;
        if (b == t) {
          for (uint32_t j = threadIdx.x; j < half; j += kT) {
            const float2 o = fma_c(lds[j], c, lds[j + half], f, 1.f);
            lds[j] = o;
            acc += n2(o);
          }
        } else {
          for (uint32_t i = threadIdx.x; i < (dim >> 2); i += kT) {
            const uint32_t j = i0(i, b), st2 = 1u << b;
            const float2 A = lds[j], B = lds[j + st2], C = lds[j + half], D = lds[j + st2 + half];
            const float2 o0 = fma_c(A, c, B, f, 1.f), o1 = fma_c(C, c, D, f, 1.f);
            lds[j] = o0;
            lds[j + st2] = o1;
            acc += n2(o0) + n2(o1);
          }
        }
      } else {
        const Window w = window_of(st);
        const float s1 = w.vw_even ? 1.f : -1.f;
        for (uint32_t i = threadIdx.x; i < (dim >> 1); i += kT) {
          const uint32_t j = i0(i, b), st2 = 1u << b;
          const float sb = (__popcll(j & w.mask_b) & 1) ? -1.f : 1.f;
          const float so1 = (__popcll(j & w.mask_o1) & 1) ? -1.f : 1.f;
          const float2 a = lds[j], bb = lds[j + st2];
          float2 o0 = fma_c(a, c, bb, f, sb), o1 = fma_c(a, c, bb, f, s1 * sb);
          if (so1 < 0.f) o1 = neg(o1);
          if (w.swap) { const float2 t = o0; o0 = o1; o1 = t; }
          if (w.neg0) o0 = neg(o0);
          if (w.neg1) o1 = neg(o1);
          lds[j] = o0;
          lds[j + st2] = o1;
          acc += n2(o0) + n2(o1);
        }
      }
      if (half) {
        if (probs && threadIdx.x == 0) probs[st.m_index] = 0.5;
        ++half_run;
      } else if (reduce != kReduceNone) {
        half_run = 0;
        const double sum = block_sum<kT>(acc, red);
        const double p = 0.5 * sum;
        if (probs && threadIdx.x == 0) probs[st.m_index] = p;
        if (reduce == kReduceRenorm) {
          if (p < 1e-10) {
            if (threadIdx.x == 0) { atomicMin(&err[0], item < 0 ? st.m_index : item); err[1] = kErrZeroProb; }
            sigma = 0.0;
          } else {
            sigma = 1.0 / sqrt(sum);
          }
        } else if (fabs(p - 0.5) > 1e-4 && threadIdx.x == 0) {
          atomicMin(&err[0], item < 0 ? st.m_index : item);
          err[1] = kErrNotDet;
        }
      }
    }
    __syncthreads();
  }
  const float scale = float((reduce == kReduceRenorm ? sigma : 1.0) * final_factor);
  const uint32_t dout = 1u << nout;
  for (uint32_t x = threadIdx.x; x < dout; x += kT) {
    uint32_t src = 0;
    for (int k = 0; k < nout; ++k) src |= ((x >> k) & 1u) << where[k];
    const float2 v = lds[src];
    out[x] = make_float2(scale * v.x, scale * v.y);
  }
  __syncthreads();
}

template <int kT>
__global__ __launch_bounds__(kT) void k_lds_batch(const LdsItem *__restrict__ items, int count) {
  extern __shared__ float2 lds[];
  __shared__ double red[kT / 64];
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    const LdsItem *x = items + it;
    run_item<kT>(x->steps, x->nsteps, x->nin, x->nout, x->where, x->final_factor, lds, x->in, x->basis, x->out,
             x->probs, x->reduce, x->err, -1, red);
  }
}

// A row of the batch table (read-only, uniform index): scalar loads.
__device__ __forceinline__ BatchIo load_io(const BatchIo *ios, uint32_t i) {
  static_assert(sizeof(BatchIo) % 4 == 0, "BatchIo is whole dwords");
  constexpr int kW = sizeof(BatchIo) / 4;
  typedef const __attribute__((address_space(4))) uint32_t cword;
  cword *src = reinterpret_cast<cword *>(reinterpret_cast<uintptr_t>(ios)) +
               size_t(kW) * __builtin_amdgcn_readfirstlane(i);
  uint32_t w[kW];
#pragma unroll
  for (int k = 0; k < kW; ++k) w[k] = src[k];
  BatchIo b;
  __builtin_memcpy(&b, w, sizeof(b));
  return b;
}

constexpr int kIoThreads = 256;

// Start of pattern blockIdx.y of a batched run: sigma = 1, its error word
// cleared, and (rows with a live vector) its input, or the empty product
// state psi[0] = 1, in the first 2^nin amplitudes of that vector.
__global__ __launch_bounds__(kIoThreads) void k_batch_start(const BatchIo *__restrict__ ios) {
  const BatchIo b = load_io(ios, blockIdx.y);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *b.book.sigma = 1.0;
    b.book.err[0] = kErrNone;
    b.book.err[1] = 0;
  }
  if (!b.psi) return;  // an LDS-resident pattern: only its error word
  const size_t n = size_t(1) << b.nin;
  for (size_t i = size_t(blockIdx.x) * kIoThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kIoThreads)
    b.psi[i] = b.in ? b.in[i] : make_float2(i == 0 ? 1.f : 0.f, 0.f);
}

// Read-out of pattern blockIdx.y: output x (bit k = outputs[k]) is the live
// amplitude at the slots where[k], times sigma and the host factor.
__global__ __launch_bounds__(kGatherThreads) void k_batch_read(const BatchIo *__restrict__ ios) {
  __shared__ uint64_t tab[1 << kGatherLo];
  const BatchIo b = load_io(ios, blockIdx.y);
  const double sg = b.reduce == kReduceRenorm ? *b.book.sigma : 1.0;
  // the slots straight from the read-only table (scalar loads)
  typedef const __attribute__((address_space(4))) int cint;
  cint *where = reinterpret_cast<cint *>(reinterpret_cast<uintptr_t>(ios + blockIdx.y) + offsetof(BatchIo, where));
  gather_chunks(b.psi, b.out, b.nout, where, float(sg * b.final_factor), tab, blockIdx.x, gridDim.x);
}

template <int kT>
__global__ __launch_bounds__(kT) void k_lds_shared(LdsItem proto, int count, int reduce, uint32_t first,
                                                    int basis_mode, size_t probs_stride) {
  extern __shared__ float2 lds[];
  __shared__ double red[kT / 64];
  const size_t din = size_t(1) << proto.nin, dout = size_t(1) << proto.nout;
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const float2 *in = basis_mode ? nullptr : proto.in + size_t(k) * din;
    double *pr = proto.probs ? proto.probs + size_t(k) * probs_stride : nullptr;
    run_item<kT>(proto.steps, proto.nsteps, proto.nin, proto.nout, proto.where, proto.final_factor, lds, in,
             basis_mode ? int(first + k) : -1, proto.out + size_t(k) * dout, pr, reduce, proto.err, k, red);
  }
}

unsigned lds_grid(int count) { return unsigned(count < 16384 ? count : 16384); }

// (the LDS limit of k_lds_batch is raised once by lds_batch_prepare, before
// any capture)
template <int kT>
hipError_t lds_batch_t(const LdsItem *items, int count, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_lds_batch<kT>, dim3(lds_grid(count)), dim3(kT), bytes, s, items, count);
  return hipGetLastError();
}

unsigned io_grid(int max_bits) {
  const size_t n = size_t(1) << max_bits;
  const size_t g = (n + kIoThreads - 1) / kIoThreads;
  return unsigned(g < 256 ? g : 256);
}

template <int kT>
hipError_t lds_shared_t(const LdsItem &proto, int count, size_t bytes, int reduce, uint32_t first, int basis_mode,
                        size_t probs_stride, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_lds_shared<kT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lds_shared<kT>, dim3(lds_grid(count)), dim3(kT), bytes, s, proto, count, reduce, first,
                     basis_mode, probs_stride);
  return hipGetLastError();
}

}  // namespace

hipError_t lds_batch_prepare() {
  const int bytes = int(sizeof(float2) << kLdsMaxWidth);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_lds_batch<64>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_lds_batch<256>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_lds_batch<512>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

hipError_t launch_lds_batch(const LdsItem *items, int count, int width, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t bytes = sizeof(float2) << width;
  switch (threads_for(width)) {
    case 64: return lds_batch_t<64>(items, count, bytes, s);
    case 256: return lds_batch_t<256>(items, count, bytes, s);
    default: return lds_batch_t<512>(items, count, bytes, s);
  }
}

hipError_t launch_batch_start(const BatchIo *ios, int count, int max_nin, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_start, dim3(io_grid(max_nin), unsigned(count)), dim3(kIoThreads), 0, s, ios);
  return hipGetLastError();
}

hipError_t launch_batch_read(const BatchIo *ios, int count, int max_nout, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // one chunk of 2^kGatherLo outputs per workgroup and trip, for the widest
  const int lo = max_nout < kGatherLo ? max_nout : kGatherLo;
  const unsigned g = unsigned(std::min<uint64_t>(uint64_t(1) << (max_nout - lo), 64));
  hipLaunchKernelGGL(k_batch_read, dim3(g, unsigned(count)), dim3(kGatherThreads), 0, s, ios);
  return hipGetLastError();
}

hipError_t launch_lds_shared(const LdsItem &proto, int count, int width, int reduce, uint32_t first,
                             int basis_mode, size_t probs_stride, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t bytes = sizeof(float2) << width;
  switch (threads_for(width)) {
    case 64: return lds_shared_t<64>(proto, count, bytes, reduce, first, basis_mode, probs_stride, s);
    case 256: return lds_shared_t<256>(proto, count, bytes, reduce, first, basis_mode, probs_stride, s);
    default: return lds_shared_t<512>(proto, count, bytes, reduce, first, basis_mode, probs_stride, s);
  }
}

}  // namespace owqs
