// owqs_gather.h -- the read-out gather shared by the single-pattern and the
// batched read kernels (device code; included by .hip files only).
//
// Output x (bit k = the k-th output qubit) is the live amplitude at
// src(x) = OR over k of (bit k of x) << where[k], times a scale.  src is
// linear over OR, so x splits into its low kGatherLo bits, whose images a
// workgroup tabulates once in LDS, and the rest, one value per chunk of
// 2^kGatherLo outputs, uniform over the workgroup (computed on the scalar
// unit).  A thread then does one LDS read and one OR per output instead of
// a loop over the output bits.
#pragma once

#include "owqs_internal.h"

namespace owqs {

constexpr int kGatherLo = 10;
constexpr int kGatherThreads = 256;
constexpr int kGatherPer = (1 << kGatherLo) / kGatherThreads;  // outputs per thread per chunk

// `where` must be uniform over the workgroup (kernel argument or a row read
// through scalar loads); tab holds 2^kGatherLo entries of LDS.
template <typename WhereT>
__device__ __forceinline__ void gather_chunks(const float2 *__restrict__ psi, float2 *__restrict__ out, int nout,
                                              const WhereT &where, float scale, uint64_t *tab, uint64_t chunk0,
                                              uint64_t chunk_step) {
  const int lo = nout < kGatherLo ? nout : kGatherLo;
  const uint32_t per_chunk = 1u << lo;
  for (uint32_t j = threadIdx.x; j < per_chunk; j += kGatherThreads) {
    uint64_t v = 0;
    for (int k = 0; k < lo; ++k) v |= uint64_t((j >> k) & 1u) << where[k];
    tab[j] = v;
  }
  __syncthreads();
  const uint64_t nchunks = uint64_t(1) << (nout - lo);
  for (uint64_t c = chunk0; c < nchunks; c += chunk_step) {
    uint64_t hi = 0;
    for (int k = lo; k < nout; ++k) hi |= ((c >> (k - lo)) & 1) << where[k];
    const uint64_t base = c << lo;
    if (per_chunk == (1u << kGatherLo)) {
      float2 v[kGatherPer];
#pragma unroll
      for (int r = 0; r < kGatherPer; ++r) v[r] = psi[hi | tab[threadIdx.x + r * kGatherThreads]];
#pragma unroll
      for (int r = 0; r < kGatherPer; ++r)
        out[base + threadIdx.x + r * kGatherThreads] = make_float2(scale * v[r].x, scale * v[r].y);
    } else {
      for (uint32_t j = threadIdx.x; j < per_chunk; j += kGatherThreads) {
        const float2 v = psi[hi | tab[j]];
        out[base + j] = make_float2(scale * v.x, scale * v.y);
      }
    }
  }
}

}  // namespace owqs
