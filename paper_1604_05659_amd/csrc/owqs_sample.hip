// owqs_sample.hip -- measurements whose outcomes are drawn on the device.
//
// The paper's simulator draws every outcome (Fig. 6): outcome 0 when a
// uniform random number does not exceed the probability of outcome 0.  Here
// the uniforms are supplied by the caller (one per M, uploaded before the
// run) and the whole decision stays on the GPU, so a run needs no host round
// trip between commands and can be replayed as a HIP graph:
//   - the signals of an M (Eq. 2) and of an X/Z correction are the XOR of
//     outcomes already drawn, read from device memory;
//   - an M is a probability pass (FP64 partial sums of the outcome-0 branch
//     and of the norm), a one-block decision that writes the outcome and the
//     collapse coefficient, then the forced-outcome collapse kernel reading
//     that coefficient, and its finishing kernel (p of the drawn outcome,
//     renormalisation).
#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ int signal_of(const int *dom, SigRef r, const int *outc) {
  int s = 0;
  for (int i = 0; i < r.len; ++i) s ^= outc[dom[r.off + i]];
  return s & 1;
}

// theta = (-1)^s alpha + t pi (Eq. 2); returns e^{-i theta} in FP64.
__device__ __forceinline__ double2 c_of(double alpha, int s, int t) {
  const double th = (s ? -alpha : alpha) + (t ? M_PI : 0.0);
  return make_double2(cos(th), -sin(th));
}

__device__ __forceinline__ uint64_t ins0(uint64_t x, int b) {
  return ((x >> b) << (b + 1)) | (x & ((uint64_t(1) << b) - 1));
}

__global__ __launch_bounds__(kB) void k_s_pauli(float2 *__restrict__ psi, uint64_t half, int b, int x, SigRef sig,
                                                 const int *__restrict__ dom, const int *__restrict__ outc) {
  if (!signal_of(dom, sig, outc)) return;  // the same for every thread
  const uint64_t bit = uint64_t(1) << b;
  for (uint64_t q = uint64_t(blockIdx.x) * kB + threadIdx.x; q < half; q += uint64_t(gridDim.x) * kB) {
    const uint64_t i0 = ins0(q, b), i1 = i0 | bit;
    const float2 v1 = psi[i1];
    if (x) {
      psi[i1] = psi[i0];
      psi[i0] = v1;
    } else {
      psi[i1] = make_float2(-v1.x, -v1.y);
    }
  }
}

__device__ void block_sum2(double a, double b, double *out_a, double *out_b) {
  __shared__ double wa[kB / 64], wb[kB / 64];
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    wa[w] = a;
    wb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < kB / 64; ++k) {
      sa += wa[k];
      sb += wb[k];
    }
    *out_a = sa;
    *out_b = sb;
  }
}

__global__ __launch_bounds__(kB) void k_s_prob(const float2 *__restrict__ psi, uint64_t half, int b, double alpha,
                                                SigRef sg, SigRef tg, const int *__restrict__ dom,
                                                const int *__restrict__ outc, double *partials) {
  const double2 cd = c_of(alpha, signal_of(dom, sg, outc), signal_of(dom, tg, outc));
  const float2 c = make_float2(float(cd.x), float(cd.y));
  const uint64_t bit = uint64_t(1) << b;
  double acc0 = 0.0, accn = 0.0;
  for (uint64_t q = uint64_t(blockIdx.x) * kB + threadIdx.x; q < half; q += uint64_t(gridDim.x) * kB) {
    const uint64_t i0 = ins0(q, b);
    const float2 a = psi[i0], v = psi[i0 | bit];
    const float ox = a.x + (c.x * v.x - c.y * v.y), oy = a.y + (c.x * v.y + c.y * v.x);
    acc0 += double(ox) * ox + double(oy) * oy;
    accn += double(a.x) * a.x + double(a.y) * a.y + double(v.x) * v.x + double(v.y) * v.y;
  }
  block_sum2(acc0, accn, partials + blockIdx.x, partials + kSampleGrid + blockIdx.x);
}

// p_0 = sum |psi_0 + c0 psi_1|^2 / (2 sum |psi|^2): the probability of
// outcome 0 whatever the current scale of the vector.
__global__ __launch_bounds__(kB) void k_s_decide(const double *__restrict__ partials, unsigned nparts,
                                                  const double *__restrict__ u, int m, double alpha, SigRef sg,
                                                  SigRef tg, const int *__restrict__ dom, int *outc, float2 *coef) {
  double a = 0.0, n = 0.0;
  for (unsigned i = threadIdx.x; i < nparts; i += kB) {  // fixed order per thread
    a += partials[i];
    n += partials[kSampleGrid + i];
  }
  __shared__ double sa, sn;
  block_sum2(a, n, &sa, &sn);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double p0 = sn > 0.0 ? 0.5 * sa / sn : 0.0;
    const int o = (sn > 0.0 && u[m] <= p0) ? 0 : 1;
    double2 c = c_of(alpha, signal_of(dom, sg, outc), signal_of(dom, tg, outc));
    if (o) c = make_double2(-c.x, -c.y);
    outc[m] = o;
    *coef = make_float2(float(c.x), float(c.y));
  }
}

__global__ void k_s_jdecide(const double *__restrict__ u, int m, double alpha, SigRef sg, SigRef tg,
                            const int *__restrict__ dom, int *outc, float2 *coef, const FoldRef *__restrict__ folds,
                            int nf, int *fold) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int o = u[m] <= 0.5 ? 0 : 1;
  double2 c = c_of(alpha, signal_of(dom, sg, outc), signal_of(dom, tg, outc));
  if (o) c = make_double2(-c.x, -c.y);
  outc[m] = o;
  *coef = make_float2(float(c.x), float(c.y));
  // the corrections on w after M v, in order, as a signed permutation
  int i0 = 0, s0 = 1, s1 = 1;
  for (int k = 0; k < nf; ++k) {
    if (!signal_of(dom, folds[k].sig, outc)) continue;
    if (folds[k].x) {
      i0 ^= 1;
      const int t = s0;
      s0 = s1;
      s1 = t;
    } else {
      s1 = -s1;
    }
  }
  fold[0] = i0;
  fold[1] = s0 < 0;
  fold[2] = s1 < 0;
}

// Every drawn window of a plan in which every M is such a window: thread i
// resolves window i.  Each outcome is (u <= 1/2 ? 0 : 1) (p = 1/2 exactly),
// so a signal (Eq. 2) is the XOR of those bits over its domain, read from the
// uniforms without waiting for any other thread.
__global__ __launch_bounds__(kB) void k_s_resolve(const DrawWin *__restrict__ wins, int nwin,
                                                   const double *__restrict__ u, const int *__restrict__ dom,
                                                   const FoldRef *__restrict__ folds, int *outc, float2 *ctab,
                                                   int *ftab, FuseOp *fops) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= nwin) return;
  const DrawWin w = wins[i];
  auto sig = [&](SigRef r) {
    int v = 0;
    for (int k = 0; k < r.len; ++k) v ^= u[dom[r.off + k]] <= 0.5 ? 0 : 1;
    return v;
  };
  const int o = u[w.m] <= 0.5 ? 0 : 1;
  double2 c = c_of(w.alpha, sig(w.s), sig(w.t));
  if (o) c = make_double2(-c.x, -c.y);
  outc[w.m] = o;
  ctab[w.m] = make_float2(float(c.x), float(c.y));
  int i0 = 0, s0 = 1, s1 = 1;  // the corrections on w as a signed permutation
  for (int k = 0; k < w.fold_len; ++k) {
    const FoldRef f = folds[w.fold_off + k];
    if (!sig(f.sig)) continue;
    if (f.x) {
      i0 ^= 1;
      const int t = s0;
      s0 = s1;
      s1 = t;
    } else {
      s1 = -s1;
    }
  }
  ftab[3 * w.m] = i0;
  ftab[3 * w.m + 1] = s0 < 0;
  ftab[3 * w.m + 2] = s1 < 0;
  if (w.fop >= 0) {  // vector stores; the next kernel's scalar loads read them after the launch boundary
    FuseOp *op = fops + w.fop;
    // the row holds the window's factor times its coefficient (as the host writes it)
    const double f = double(op->f);
    op->coef = make_float2(float(f * double(float(c.x))), float(f * double(float(c.y))));
    op->flags = uint8_t((op->flags & ~7u) | uint32_t(i0) | (s0 < 0 ? 2u : 0u) | (s1 < 0 ? 4u : 0u));
    round_words(*op);
  }
}

unsigned grid_of(uint64_t units) {
  uint64_t g = (units + kB - 1) / kB;
  if (g < 1) g = 1;
  if (g > kSampleGrid) g = kSampleGrid;
  return unsigned(g);
}

}  // namespace

hipError_t launch_s_pauli(float2 *psi, int n, int b, int x, SigRef sig, const int *dom, const int *outc,
                          hipStream_t s) {
  const uint64_t half = (uint64_t(1) << n) >> 1;
  hipLaunchKernelGGL(k_s_pauli, dim3(grid_of(half)), dim3(kB), 0, s, psi, half, b, x, sig, dom, outc);
  return hipGetLastError();
}

hipError_t launch_s_prob(const float2 *psi, int n, int b, double alpha, SigRef sg, SigRef tg, const int *dom,
                         const int *outc, double *partials, unsigned *grid, hipStream_t s) {
  const uint64_t half = (uint64_t(1) << n) >> 1;
  const unsigned g = grid_of(half);
  hipLaunchKernelGGL(k_s_prob, dim3(g), dim3(kB), 0, s, psi, half, b, alpha, sg, tg, dom, outc, partials);
  *grid = g;
  return hipGetLastError();
}

hipError_t launch_s_decide(const double *partials, unsigned nparts, const double *u, int m, double alpha,
                           SigRef sg, SigRef tg, const int *dom, int *outc, float2 *coef, hipStream_t s) {
  hipLaunchKernelGGL(k_s_decide, dim3(1), dim3(kB), 0, s, partials, nparts, u, m, alpha, sg, tg, dom, outc, coef);
  return hipGetLastError();
}

hipError_t launch_s_jdecide(const double *u, int m, double alpha, SigRef sg, SigRef tg, const int *dom, int *outc,
                            float2 *coef, const FoldRef *folds, int nf, int *fold, hipStream_t s) {
  hipLaunchKernelGGL(k_s_jdecide, dim3(1), dim3(64), 0, s, u, m, alpha, sg, tg, dom, outc, coef, folds, nf, fold);
  return hipGetLastError();
}

namespace {

// Composed maps of a drawn run (one thread per map): the product of its
// windows' maps from the rows k_s_resolve has just written, as the plan
// compiler forms it for forced outcomes.  refs[off[i] ..]: the map's row in
// mrows, its window count, its windows' rows in fops.
__global__ __launch_bounds__(kB) void k_s_compose(const FuseOp *__restrict__ fops, FuseOp *__restrict__ mrows,
                                                   const int *__restrict__ refs, const int *__restrict__ off,
                                                   int nmaps) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= nmaps) return;
  const int *r = refs + off[i];
  const int row = r[0], cnt = r[1];
  double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  for (int c = 0; c < cnt; ++c) {
    double w[8];
    window_map(fops[r[2 + c]], w);
    map_left(w, u);
  }
  FuseOp m = mrows[row];
  map_store(m, u);
  mrows[row] = m;
}

}  // namespace

hipError_t launch_s_compose(const FuseOp *fops, FuseOp *mrows, const int *refs, const int *off, int nmaps,
                            hipStream_t s) {
  if (nmaps <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_s_compose, dim3(unsigned((nmaps + kB - 1) / kB)), dim3(kB), 0, s, fops, mrows, refs, off,
                     nmaps);
  return hipGetLastError();
}

hipError_t launch_s_resolve(const DrawWin *wins, int nwin, const double *u, const int *dom, const FoldRef *folds,
                            int *outc, float2 *ctab, int *ftab, FuseOp *fops, hipStream_t s) {
  if (nwin <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_s_resolve, dim3(unsigned((nwin + kB - 1) / kB)), dim3(kB), 0, s, wins, nwin, u, dom, folds,
                     outc, ctab, ftab, fops);
  return hipGetLastError();
}

}  // namespace owqs
