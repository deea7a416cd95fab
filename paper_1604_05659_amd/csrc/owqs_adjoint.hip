// owqs_adjoint.hip -- batched forward and adjoint sweeps for the gradient of
// an output observable with respect to the measurement angles.
//
// B angle sets of one pattern run side by side: the state buffer holds B
// vectors of `stride` amplitudes each, and every kernel takes the set as
// blockIdx.y.  The plan is the fused one: after a prefix without parameters
// (preparations), every step is a window (N w; E u w; M u; X/Z on w) or a
// Pauli / controlled-Z step.  With fixed probability 1/2 (Sec. 4.5) a window
// is, at every index j of the other slots, the unitary (up to the factor f)
// P diag(1, so1) f [[1, c sb], [1, s c sb]] on one slot (f = 1/sqrt 2, c =
// (-1)^o e^{-i theta}, Eqs. 11-12; sb, so1, s the signs of the E commands
// inside the window; P the folded corrections), and E, X, Z are self-adjoint,
// so the reverse sweep carries the adjoint state
// lambda = U_{>k}^dagger (W psi_final) back through the windows:
//   dL/dtheta_k = 2 Re <lambda_k | dW_k/dtheta psi_{k-1}>,
// and dtheta/dalpha = (-1)^s (Eq. 2).  Gradient partials are FP64 per block;
// one reduction kernel sums them in block order at the end.
#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ uint64_t j0(uint64_t x, int b) {
  return ((x >> b) << (b + 1)) | (x & ((uint64_t(1) << b) - 1));
}
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

#define SET_LOOP(count)                                                                          \
  float2 *const v = psi + size_t(blockIdx.y) * stride;                                            \
  for (uint64_t i = uint64_t(blockIdx.x) * kB + threadIdx.x; i < (count); i += uint64_t(gridDim.x) * kB)

// Every set starts from the same input: in[0 .. din), or the empty product
// state (the single amplitude 1) when in is null (then din = 1).
__global__ __launch_bounds__(kB) void k_b_init(float2 *psi, size_t stride, uint64_t din, const float2 *in) {
  SET_LOOP(din) v[i] = in ? in[i] : make_float2(i == 0 ? 1.f : 0.f, 0.f);
}

__global__ __launch_bounds__(kB) void k_b_prepare(float2 *psi, size_t stride, uint64_t dim) {
  SET_LOOP(dim) v[i + dim] = v[i];
}

__global__ __launch_bounds__(kB) void k_b_cz(float2 *psi, size_t stride, uint64_t quarter, int lo, int hi) {
  SET_LOOP(quarter) {
    const uint64_t j = j0(j0(i, lo), hi) | (uint64_t(1) << lo) | (uint64_t(1) << hi);
    v[j] = make_float2(-v[j].x, -v[j].y);
  }
}

__global__ __launch_bounds__(kB) void k_b_x(float2 *psi, size_t stride, uint64_t half, int b) {
  SET_LOOP(half) {
    const uint64_t j = j0(i, b), k = j | (uint64_t(1) << b);
    const float2 t = v[j];
    v[j] = v[k];
    v[k] = t;
  }
}

__global__ __launch_bounds__(kB) void k_b_z(float2 *psi, size_t stride, uint64_t half, int b) {
  SET_LOOP(half) {
    const uint64_t j = j0(i, b) | (uint64_t(1) << b);
    v[j] = make_float2(-v[j].x, -v[j].y);
  }
}

__device__ __forceinline__ float sgnb(uint64_t j, uint64_t mask) { return (__popcll(j & mask) & 1) ? -1.f : 1.f; }

// Forward window on every set (see Window): o0 = f (a + c sb b),
// o1 = so1 f (a + s c sb b), then the folded corrections.
__global__ __launch_bounds__(kB) void k_b_window(float2 *psi, size_t stride, uint64_t half, int b,
                                                  const float2 *coefs, float f, Window w) {
  const float2 c = coefs[blockIdx.y];
  const float s1 = w.vw_even ? 1.f : -1.f;
  SET_LOOP(half) {
    const uint64_t j = j0(i, b), k = j | (uint64_t(1) << b);
    const float sb = sgnb(j, w.mask_b), so1 = sgnb(j, w.mask_o1);
    const float2 a = v[j], cb0 = cmulf(c, v[k]);
    const float2 cb = make_float2(sb * cb0.x, sb * cb0.y);
    float2 o0 = make_float2(f * (a.x + cb.x), f * (a.y + cb.y));
    float2 o1 = make_float2(so1 * f * (a.x + s1 * cb.x), so1 * f * (a.y + s1 * cb.y));
    if (w.swap) { const float2 t = o0; o0 = o1; o1 = t; }
    if (w.neg0) o0 = make_float2(-o0.x, -o0.y);
    if (w.neg1) o1 = make_float2(-o1.x, -o1.y);
    v[j] = o0;
    v[k] = o1;
  }
}

// Adjoint of one window: psi_in = the window's input (read only), lam = the
// adjoint state after the window (updated in place to the state before it).
// With mu = P^T lam (P the folded corrections):
//   d(o0, o1)/dtheta = P (f sb (-i c b), so1 s f sb (-i c b)),
//   lam_a = f (mu0 + so1 mu1),  lam_b = f sb conj(c) (mu0 + so1 s mu1).
// partials[set * gridDim.x + block] = this block's sum of
// 2 Re <lam | dW/dtheta psi_in>.
__global__ __launch_bounds__(kB) void k_b_window_adj(const float2 *__restrict__ psi_in, float2 *__restrict__ lam,
                                                      size_t stride, uint64_t half, int b, const float2 *coefs,
                                                      float f, Window w, double *partials) {
  __shared__ double red[kB / 64];
  const float2 c = coefs[blockIdx.y];
  const float s1 = w.vw_even ? 1.f : -1.f;
  const float2 *x = psi_in + size_t(blockIdx.y) * stride;
  float2 *l = lam + size_t(blockIdx.y) * stride;
  double acc = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * kB + threadIdx.x; i < half; i += uint64_t(gridDim.x) * kB) {
    const uint64_t j = j0(i, b), k = j | (uint64_t(1) << b);
    const float sb = sgnb(j, w.mask_b), so1 = sgnb(j, w.mask_o1);
    const float2 cb = cmulf(c, x[k]);                                   // c b
    // -i c b = (cb.y, -cb.x)
    const float g0 = f * sb, g1 = so1 * s1 * f * sb;
    float2 d0 = make_float2(g0 * cb.y, -g0 * cb.x), d1 = make_float2(g1 * cb.y, -g1 * cb.x);
    if (w.swap) { const float2 t = d0; d0 = d1; d1 = t; }
    if (w.neg0) d0 = make_float2(-d0.x, -d0.y);
    if (w.neg1) d1 = make_float2(-d1.x, -d1.y);
    const float2 l0 = l[j], l1 = l[k];
    acc += 2.0 * (double(l0.x) * d0.x + double(l0.y) * d0.y + double(l1.x) * d1.x + double(l1.y) * d1.y);
    // mu = P^T lam: undo the negations, then the swap
    float2 m0 = w.neg0 ? make_float2(-l0.x, -l0.y) : l0;
    float2 m1 = w.neg1 ? make_float2(-l1.x, -l1.y) : l1;
    if (w.swap) { const float2 t = m0; m0 = m1; m1 = t; }
    const float2 sm = make_float2(m0.x + so1 * m1.x, m0.y + so1 * m1.y);
    const float2 dm = make_float2(m0.x + so1 * s1 * m1.x, m0.y + so1 * s1 * m1.y);
    const float2 cd = cmulf(make_float2(c.x, -c.y), dm);
    l[j] = make_float2(f * sm.x, f * sm.y);
    l[k] = make_float2(f * sb * cd.x, f * sb * cd.y);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kB / 64; ++q) t += red[q];
    partials[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

// Reverse sweep through one window whose 2x2 part is invertible (an odd
// number of E between its two qubits, s = -1): with K = [[1, sb c], [1, -sb c]]
// and |c| = 1, K^dagger K = 2, so the window's input is recovered from its
// output as psi_in = (1 / (2 f^2)) W^dagger psi_out, the same map the adjoint
// state takes (up to the scale).  One pass reads psi_out and lam_out, writes
// psi_in and lam_in, and adds this block's 2 Re <lam | dW/dtheta psi_in> to
// partials[set * prow + block] (see k_b_window_adj; prow >= gridDim.x).
__global__ __launch_bounds__(kB) void k_b_window_rev(float2 *__restrict__ psi, float2 *__restrict__ lam,
                                                      size_t stride, uint64_t half, int b, const float2 *coefs,
                                                      float f, Window w, double *partials, unsigned prow) {
  __shared__ double red[kB / 64];
  const float2 c = coefs[blockIdx.y];
  const float2 cc = make_float2(c.x, -c.y);
  const float g = 0.5f / f;
  float2 *x = psi + size_t(blockIdx.y) * stride;
  float2 *l = lam + size_t(blockIdx.y) * stride;
  double acc = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * kB + threadIdx.x; i < half; i += uint64_t(gridDim.x) * kB) {
    const uint64_t j = j0(i, b), k = j | (uint64_t(1) << b);
    const float sb = sgnb(j, w.mask_b), so1 = sgnb(j, w.mask_o1);
    // undo the folded corrections on the output, then invert K
    float2 o0 = x[j], o1 = x[k];
    if (w.neg0) o0 = make_float2(-o0.x, -o0.y);
    if (w.neg1) o1 = make_float2(-o1.x, -o1.y);
    if (w.swap) { const float2 t = o0; o0 = o1; o1 = t; }
    const float2 pa = make_float2(g * (o0.x + so1 * o1.x), g * (o0.y + so1 * o1.y));
    const float2 pd = cmulf(cc, make_float2(o0.x - so1 * o1.x, o0.y - so1 * o1.y));
    const float2 pb = make_float2(g * sb * pd.x, g * sb * pd.y);
    // gradient term with the recovered input (s = -1)
    const float2 cb = cmulf(c, pb);
    const float g0 = f * sb, g1 = -so1 * f * sb;
    float2 d0 = make_float2(g0 * cb.y, -g0 * cb.x), d1 = make_float2(g1 * cb.y, -g1 * cb.x);
    if (w.swap) { const float2 t = d0; d0 = d1; d1 = t; }
    if (w.neg0) d0 = make_float2(-d0.x, -d0.y);
    if (w.neg1) d1 = make_float2(-d1.x, -d1.y);
    const float2 l0 = l[j], l1 = l[k];
    acc += 2.0 * (double(l0.x) * d0.x + double(l0.y) * d0.y + double(l1.x) * d1.x + double(l1.y) * d1.y);
    float2 m0 = w.neg0 ? make_float2(-l0.x, -l0.y) : l0;
    float2 m1 = w.neg1 ? make_float2(-l1.x, -l1.y) : l1;
    if (w.swap) { const float2 t = m0; m0 = m1; m1 = t; }
    const float2 sm = make_float2(m0.x + so1 * m1.x, m0.y + so1 * m1.y);
    const float2 cd = cmulf(cc, make_float2(m0.x - so1 * m1.x, m0.y - so1 * m1.y));
    x[j] = pa;
    x[k] = pb;
    l[j] = make_float2(f * sm.x, f * sm.y);
    l[k] = make_float2(f * sb * cd.x, f * sb * cd.y);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kB / 64; ++q) t += red[q];
    partials[size_t(blockIdx.y) * prow + blockIdx.x] = t;
  }
}

struct ObsBits {
  int n;
  int bit[kWhereMax];
};

// Loss L = ff2 * sum_x W(x) |psi(x)|^2, W(x) = sum_k (1 - 2 bit_{obs_k}(x));
// lam = ff2 * W * psi.  partials[set * gridDim.x + block].
__global__ __launch_bounds__(kB) void k_b_loss(const float2 *__restrict__ psi, float2 *__restrict__ lam,
                                                size_t stride, uint64_t dim, ObsBits ob, double ff2,
                                                double *partials) {
  __shared__ double red[kB / 64];
  const float2 *x = psi + size_t(blockIdx.y) * stride;
  float2 *l = lam + size_t(blockIdx.y) * stride;
  double acc = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * kB + threadIdx.x; i < dim; i += uint64_t(gridDim.x) * kB) {
    int wsum = 0;
    for (int k = 0; k < ob.n; ++k) wsum += 1 - 2 * int((i >> ob.bit[k]) & 1);
    const float2 a = x[i];
    acc += ff2 * wsum * (double(a.x) * a.x + double(a.y) * a.y);
    const float w = float(ff2 * wsum);
    l[i] = make_float2(w * a.x, w * a.y);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kB / 64; ++q) t += red[q];
    partials[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

// out[r * out_stride + out_col[q]] = scale[q] * sum of partials[r][q][0..nblk)
// for rows r (sets) and columns q (windows); one thread per (r, q).
__global__ __launch_bounds__(kB) void k_b_reduce(const double *__restrict__ partials, int nq, int nsets, int nblk,
                                                  const int *out_col, const double *scale, double *out,
                                                  size_t out_stride) {
  const int id = blockIdx.x * kB + threadIdx.x;
  if (id >= nq * nsets) return;
  const int q = id / nsets, r = id % nsets;
  const double *p = partials + (size_t(q) * nsets + r) * nblk;
  double t = 0.0;
  for (int k = 0; k < nblk; ++k) t += p[k];
  out[size_t(r) * out_stride + out_col[q]] = scale[q] * t;
}

unsigned blocks_for(uint64_t count) {
  uint64_t g = (count + kB - 1) / kB;
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return unsigned(g);
}

}  // namespace

hipError_t launch_b_step(const DevStep &st, float2 *psi, size_t stride, int nsets, const float2 *coefs,
                         hipStream_t s) {
  const uint64_t dim = uint64_t(1) << st.n;
  switch (st.kind) {
    case DK_N:
      hipLaunchKernelGGL(k_b_prepare, dim3(blocks_for(dim), nsets), dim3(kB), 0, s, psi, stride, dim);
      break;
    case DK_E: {
      const int lo = st.b0 < st.b1 ? st.b0 : st.b1, hi = st.b0 < st.b1 ? st.b1 : st.b0;
      hipLaunchKernelGGL(k_b_cz, dim3(blocks_for(dim >> 2), nsets), dim3(kB), 0, s, psi, stride, dim >> 2, lo, hi);
      break;
    }
    case DK_X:
      hipLaunchKernelGGL(k_b_x, dim3(blocks_for(dim >> 1), nsets), dim3(kB), 0, s, psi, stride, dim >> 1,
                         int(st.b0));
      break;
    case DK_Z:
      hipLaunchKernelGGL(k_b_z, dim3(blocks_for(dim >> 1), nsets), dim3(kB), 0, s, psi, stride, dim >> 1,
                         int(st.b0));
      break;
    case DK_J:
      hipLaunchKernelGGL(k_b_window, dim3(blocks_for(dim >> 1), nsets), dim3(kB), 0, s, psi, stride, dim >> 1,
                         int(st.b0), coefs, st.host_factor, window_of(st));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_b_init(float2 *psi, size_t stride, int nsets, int nin, const float2 *in, hipStream_t s) {
  const uint64_t din = uint64_t(1) << nin;
  hipLaunchKernelGGL(k_b_init, dim3(blocks_for(din), nsets), dim3(kB), 0, s, psi, stride, din, in);
  return hipGetLastError();
}

unsigned adj_blocks(int n) { return blocks_for((uint64_t(1) << n) >> 1); }

hipError_t launch_b_window_adj(const DevStep &st, const float2 *psi_in, float2 *lam, size_t stride, int nsets,
                               const float2 *coefs, double *partials, hipStream_t s) {
  const uint64_t half = (uint64_t(1) << st.n) >> 1;
  hipLaunchKernelGGL(k_b_window_adj, dim3(blocks_for(half), nsets), dim3(kB), 0, s, psi_in, lam, stride, half,
                     int(st.b0), coefs, st.host_factor, window_of(st), partials);
  return hipGetLastError();
}

hipError_t launch_b_window_rev(const DevStep &st, float2 *psi, float2 *lam, size_t stride, int nsets,
                               const float2 *coefs, double *partials, unsigned prow, hipStream_t s) {
  const uint64_t half = (uint64_t(1) << st.n) >> 1;
  const unsigned g = blocks_for(half);
  if (g > prow) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_b_window_rev, dim3(g, nsets), dim3(kB), 0, s, psi, lam, stride, half, int(st.b0), coefs,
                     st.host_factor, window_of(st), partials, prow);
  return hipGetLastError();
}

unsigned loss_blocks(int n) { return blocks_for(uint64_t(1) << n); }

hipError_t launch_b_loss(const float2 *psi, float2 *lam, size_t stride, int nsets, int n, const int *obs_bits,
                         int nobs, double ff2, double *partials, hipStream_t s) {
  ObsBits ob{};
  ob.n = nobs;
  for (int k = 0; k < nobs; ++k) ob.bit[k] = obs_bits[k];
  const uint64_t dim = uint64_t(1) << n;
  hipLaunchKernelGGL(k_b_loss, dim3(blocks_for(dim), nsets), dim3(kB), 0, s, psi, lam, stride, dim, ob, ff2,
                     partials);
  return hipGetLastError();
}

hipError_t launch_b_reduce(const double *partials, int nq, int nsets, int nblk, const int *out_col,
                           const double *scale, double *out, size_t out_stride, hipStream_t s) {
  const int n = nq * nsets;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_reduce, dim3((n + kB - 1) / kB), dim3(kB), 0, s, partials, nq, nsets, nblk, out_col, scale,
                     out, out_stride);
  return hipGetLastError();
}

}  // namespace owqs
