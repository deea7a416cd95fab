// owqs_internal.h -- declarations shared by the host plan compiler and the
// gfx950 kernels of libowqs.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace owqs {

// Device-resident bookkeeping of one pattern run.
struct DevBook {
  double *sigma;      // [1] FP64 scale: true state = sigma * host factor * stored vector
  double *probs;      // [n_meas] FP64 outcome probability of every M
  double *partials;   // [kMaxPartials] per-block partial sums of |out|^2
  int *err;           // [2] {first failing M index or INT_MAX, error kind}
};

constexpr int kMaxPartials = 1 << 16;
constexpr int kWhereMax = 40;     // >= OWQS_MAX_WIDTH
constexpr int kErrNone = 0x7fffffff;
constexpr int kErrZeroProb = 1;
constexpr int kErrNotDet = 2;

// How a measurement-type kernel finishes: reduce |out|^2 in FP64 or not.
enum ReduceMode : int {
  kReduceNone = 0,      // EOWQS: no probability computed
  kReduceRenorm = 1,    // OWQS: p recorded, sigma <- 1/||out||
  kReduceCheck = 2      // EOWQS check: p recorded and compared with 1/2
};

struct MeasureArgs {
  float2 coef;          // (-1)^o e^{-i theta} rounded to complex64
  double host_factor;   // (1/sqrt 2)^(N commands since the previous M)
  int reduce;           // ReduceMode
  int m_index;          // index of this M (probs slot)
  DevBook book;
};

// Signed 2x2 permutation applied to a window's two outputs (X/Z on the new
// qubit folded in): first swap if `swap`, then negate entry 0 / entry 1.
struct PostPerm {
  int swap, neg0, neg1;
};

// ---- launchers (owqs_kernels.hip); all enqueue on `s` and return the launch status
// Reset the book (sigma = 1, no error); with set_one also psi[0] = 1
// (the empty product state when the pattern has no inputs).
hipError_t launch_init(float2 *psi, DevBook book, hipStream_t s, int set_one);
hipError_t launch_prepare(float2 *psi, int n, hipStream_t s);
hipError_t launch_cz(float2 *psi, int n, int b0, int b1, hipStream_t s);
hipError_t launch_pauli_x(float2 *psi, int n, int b, hipStream_t s);
hipError_t launch_pauli_z(float2 *psi, int n, int b, hipStream_t s);
// M and the window: the streaming kernel (writes one FP64 partial per block
// unless the mode skips probabilities); *grid receives its block count.
// launch_finish then reduces the partials (no-op when the mode skips them).
hipError_t launch_measure(float2 *psi, int n, int b, const MeasureArgs &a, hipStream_t s, unsigned *grid);
hipError_t launch_jwindow(float2 *psi, int n, int b, const MeasureArgs &a, PostPerm pp, hipStream_t s,
                          unsigned *grid);
hipError_t launch_finish(const MeasureArgs &a, unsigned nparts, hipStream_t s);
hipError_t launch_read(const float2 *psi, float2 *out, int nout, const int *where, double host_factor,
                       const double *sigma, hipStream_t s);

}  // namespace owqs
