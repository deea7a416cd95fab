// owqs_substate.hip -- kernels of the sub-state executor (Sec. 4.1).
//
// The state is a tensor product of sub-states, each in its own vector (a
// "chain": one region of an arena, grown in place).  An E across two
// sub-states first forms their tensor product (Sec. 4.4.1).  The merge runs
// in place in the wider sub-state's region: with A (a qubits, lower bits) and
// B (b qubits, upper bits),
//   C[i + 2^a j] = A[i] B[j],   0 <= i < 2^a, 0 <= j < 2^b.
// The blocks j >= 1 lie outside A's region and are written in parallel over
// (j, i) by one kernel, which only reads A; a second kernel then scales A's
// own block by B[0].  The kernel boundary is the only ordering needed.  The
// sub-state scales multiply as well: sigma_C = sigma_A sigma_B (FP64).
//
// The other commands of the executor reuse the single-vector kernels on a
// sub-state's region with that sub-state's scale (see owqs_host.cpp).
#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kB = 256;
constexpr unsigned kCap = 4096;
constexpr int kOwnUnitsLog2 = 19;  // 2^19 units of A: enough threads to stream the product alone

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Every sub-state scale to 1 and the error word cleared (start of a run).
__global__ void k_sub_start(double *sigma, int nchains, int *err) {
  for (int i = threadIdx.x; i < nchains; i += blockDim.x) sigma[i] = 1.0;
  if (threadIdx.x == 0) {
    err[0] = kErrNone;
    err[1] = 0;
  }
}

// A new sub-state holding no qubit yet: the scalar 1.
__global__ void k_sub_init(float2 *psi) {
  if (threadIdx.x == 0) psi[0] = make_float2(1.f, 0.f);
}

// In-place tensor product, a >= 1, first kernel: the blocks j >= 1,
// C[i + 2^a j] = A[i] B[j], written outside A's region (which is only read).
// A unit is two amplitudes of one block; consecutive threads take
// consecutive units, so the stores of a wave are contiguous.  A is re-read
// once per block j (from cache: it is the smaller read stream).
__global__ __launch_bounds__(kB) void k_kron_hi(float2 *__restrict__ base, uint64_t units, int ah, int a,
                                                const float2 *__restrict__ top) {
  const uint64_t mask = (uint64_t(1) << ah) - 1;
  for (uint64_t t = uint64_t(blockIdx.x) * (2 * kB) + threadIdx.x; t < units; t += uint64_t(gridDim.x) * (2 * kB)) {
    const uint64_t t1 = t + kB;
    const uint64_t u0 = t & mask, j0 = 1 + (t >> ah);
    const uint64_t u1 = t1 & mask, j1 = 1 + (t1 >> ah);
    const bool has1 = t1 < units;
    const float4 v0 = *reinterpret_cast<const float4 *>(base + 2 * u0);
    const float2 c0 = top[j0];
    float4 v1 = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 c1 = make_float2(0.f, 0.f);
    if (has1) {
      v1 = *reinterpret_cast<const float4 *>(base + 2 * u1);
      c1 = top[j1];
    }
    const float2 p00 = cmul(make_float2(v0.x, v0.y), c0), p01 = cmul(make_float2(v0.z, v0.w), c0);
    *reinterpret_cast<float4 *>(base + 2 * u0 + (j0 << a)) = make_float4(p00.x, p00.y, p01.x, p01.y);
    if (has1) {
      const float2 p10 = cmul(make_float2(v1.x, v1.y), c1), p11 = cmul(make_float2(v1.z, v1.w), c1);
      *reinterpret_cast<float4 *>(base + 2 * u1 + (j1 << a)) = make_float4(p10.x, p10.y, p11.x, p11.y);
    }
  }
}

// Wide A (2^(a-1) units fill the chip by themselves): one kernel, each
// thread owning a unit of A.  It reads the unit once, writes its products
// with B[1 .. 2^b) (outside A's region, which no thread writes yet), and last
// overwrites the unit with its product with B[0]; no other thread reads it.
__global__ __launch_bounds__(kB) void k_kron_own(float2 *__restrict__ base, uint64_t units, int a,
                                                 const float2 *__restrict__ top, uint64_t ntop, double *sig_a,
                                                 const double *sig_b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *sig_a = *sig_a * *sig_b;  // no thread here reads sig_a
  for (uint64_t u = uint64_t(blockIdx.x) * kB + threadIdx.x; u < units; u += uint64_t(gridDim.x) * kB) {
    const float4 v = *reinterpret_cast<const float4 *>(base + 2 * u);
    const float2 v0 = make_float2(v.x, v.y), v1 = make_float2(v.z, v.w);
    for (uint64_t j = 1; j < ntop; ++j) {
      const float2 c = top[j];
      const float2 p0 = cmul(v0, c), p1 = cmul(v1, c);
      *reinterpret_cast<float4 *>(base + 2 * u + (j << a)) = make_float4(p0.x, p0.y, p1.x, p1.y);
    }
    const float2 c = top[0];
    const float2 p0 = cmul(v0, c), p1 = cmul(v1, c);
    *reinterpret_cast<float4 *>(base + 2 * u) = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
}

// Second kernel (after the first on the same stream): block j = 0 in place,
// A[i] B[0], and sigma_A *= sigma_B.
__global__ __launch_bounds__(kB) void k_kron_lo(float2 *__restrict__ base, uint64_t units,
                                                const float2 *__restrict__ top, double *sig_a, const double *sig_b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *sig_a = *sig_a * *sig_b;  // no thread here reads sig_a
  const float2 c = top[0];
  for (uint64_t u = uint64_t(blockIdx.x) * kB + threadIdx.x; u < units; u += uint64_t(gridDim.x) * kB) {
    const float4 v = *reinterpret_cast<const float4 *>(base + 2 * u);
    const float2 p0 = cmul(make_float2(v.x, v.y), c), p1 = cmul(make_float2(v.z, v.w), c);
    *reinterpret_cast<float4 *>(base + 2 * u) = make_float4(p0.x, p0.y, p1.x, p1.y);
  }
}

// v[0] = v[0] v[1] ... v[count-1] (the scalars of sub-states whose qubits
// were all measured), in index order.
__global__ void k_cprod(float2 *v, int count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double re = 1.0, im = 0.0;
  for (int i = 0; i < count; ++i) {
    const double xr = v[i].x, xi = v[i].y;
    const double r = re * xr - im * xi;
    im = re * xi + im * xr;
    re = r;
  }
  v[0] = make_float2(float(re), float(im));
}

// out[x] = scalar * prod_f F_f[pext(x, mask_f)]: the factors were read out
// with their qubits in output order, so gathering the bits of x that belong
// to factor f gives its index.
__global__ __launch_bounds__(kB) void k_assemble(float2 *__restrict__ out, uint64_t count,
                                                 const float2 *__restrict__ stage, AssembleArgs a) {
  const float2 sc = stage[a.scalar_off];
  for (uint64_t x = uint64_t(blockIdx.x) * kB + threadIdx.x; x < count; x += uint64_t(gridDim.x) * kB) {
    float2 acc = sc;
    for (int f = 0; f < a.nf; ++f) {
      const uint64_t m = a.mask[f];
      uint64_t idx = 0;
      int j = 0;
      for (int k = 0; k < 64; ++k) {
        if (!((m >> k) & 1)) continue;
        idx |= ((x >> k) & 1) << j;
        ++j;
      }
      acc = cmul(acc, stage[a.off[f] + idx]);
    }
    out[x] = acc;
  }
}

unsigned grid_of(uint64_t n) {
  uint64_t g = (n + kB - 1) / kB;
  if (g < 1) g = 1;
  if (g > kCap) g = kCap;
  return unsigned(g);
}

}  // namespace

hipError_t launch_sub_start(double *sigma, int nchains, int *err, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_start, dim3(1), dim3(kB), 0, s, sigma, nchains, err);
  return hipGetLastError();
}

hipError_t launch_sub_init(float2 *psi, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_init, dim3(1), dim3(64), 0, s, psi);
  return hipGetLastError();
}

hipError_t launch_kron(float2 *base, int a, const float2 *top, int b, double *sig_a, const double *sig_b,
                       hipStream_t s) {
  if (a < 1 || b < 1 || a + b > kWhereMax) return hipErrorInvalidValue;
  const uint64_t lo = uint64_t(1) << (a - 1);              // units of block 0
  if (a - 1 >= kOwnUnitsLog2) {
    hipLaunchKernelGGL(k_kron_own, dim3(grid_of(lo)), dim3(kB), 0, s, base, lo, a, top, uint64_t(1) << b, sig_a,
                       sig_b);
    return hipGetLastError();
  }
  const uint64_t hi = lo * ((uint64_t(1) << b) - 1);       // units of blocks 1 .. 2^b - 1
  uint64_t g = (hi + 2 * kB - 1) / (2 * kB);
  if (g > kCap) g = kCap;
  hipLaunchKernelGGL(k_kron_hi, dim3(unsigned(g)), dim3(kB), 0, s, base, hi, a - 1, a, top);
  hipLaunchKernelGGL(k_kron_lo, dim3(grid_of(lo)), dim3(kB), 0, s, base, lo, top, sig_a, sig_b);
  return hipGetLastError();
}

hipError_t launch_cprod(float2 *v, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_cprod, dim3(1), dim3(64), 0, s, v, count);
  return hipGetLastError();
}

hipError_t launch_assemble(float2 *out, int nout, const float2 *stage, const AssembleArgs &a, hipStream_t s) {
  if (a.nf < 0 || a.nf > kMaxFactors) return hipErrorInvalidValue;
  const uint64_t count = uint64_t(1) << nout;
  hipLaunchKernelGGL(k_assemble, dim3(grid_of(count)), dim3(kB), 0, s, out, count, stage, a);
  return hipGetLastError();
}

}  // namespace owqs
