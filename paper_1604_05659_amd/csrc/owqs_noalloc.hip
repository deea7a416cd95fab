// owqs_noalloc.hip -- owqs_run_noalloc: a run of a loaded pattern whose
// working memory is a fixed device array of the library, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops
// that forbid hipMalloc).
//
// The run is the one owqs_run makes (Sec. 2.2 commands with qubit elimination,
// Sec. 4.2; the same kernels in the same order), with the live vector, the
// FP64 scale, the block partials, the error word and the probabilities placed
// in `scratch` instead of the pattern's own buffers.  The pattern's command
// table (uploaded by an earlier owqs_run) is only read.
#include <mutex>

#include "owqs_host_impl.h"

namespace {

using owqs::kMaxPartials;

constexpr int kNaMaxWidth = OWQS_NOALLOC_MAX_WIDTH;
constexpr size_t kNaMaxMeas = size_t(1) << 16;
// Layout: sigma (8 B) and the error word (8 B) in the first 256 bytes, then
// the block partials, the probabilities and the live vector.
constexpr size_t kOffSigma = 0;
constexpr size_t kOffErr = 16;
constexpr size_t kOffPartials = 256;
constexpr size_t kOffProbs = kOffPartials + size_t(kMaxPartials) * sizeof(double);
constexpr size_t kOffPsi = kOffProbs + kNaMaxMeas * sizeof(double);
constexpr size_t kScratchBytes = kOffPsi + (size_t(1) << kNaMaxWidth) * sizeof(float2);
static_assert(kOffPsi % 256 == 0, "the live vector starts 256-byte aligned");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];  // device address of `scratch` on each device

}  // namespace

// The working memory of owqs_run_noalloc (about 34 MiB on every device the
// library runs on, held until the process ends).  In host code this name is a
// host-side stand-in: kernels get the device address resolved below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace owqs {

hipError_t noalloc_scratch(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_addr[device] = ptr;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace owqs

extern "C" owqs_status owqs_run_noalloc(owqs_pattern *p, const void *input, size_t n_in_amps, void *output,
                                        size_t n_out_amps, double *probs, int32_t *err, void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  owqs_ctx *ctx = p->ctx;
  if (p->max_live > kNaMaxWidth)
    return fail(ctx, OWQS_E_WIDTH, "live width " + std::to_string(p->max_live) +
                                       " above the allocation-free limit " + std::to_string(kNaMaxWidth));
  if (!probs && size_t(p->n_meas) > kNaMaxMeas)
    return fail(ctx, OWQS_E_WIDTH, "more than 65536 M commands: pass a probability buffer");
  if (substates(p)) return refuse_substates(p, "owqs_run_noalloc");
  if (p->sampling) return fail(ctx, OWQS_E_STATE, "owqs_run_noalloc takes forced outcomes (uniforms are set)");
  const size_t nin = p->inputs.size(), nout = p->outputs.size();
  if (n_in_amps != (size_t(1) << nin)) return fail(ctx, OWQS_E_INVALID_ARG, "input size must be 2^(inputs)");
  if (nin > 0 && !input) return fail(ctx, OWQS_E_INVALID_ARG, "null input");
  if (!output || n_out_amps != (size_t(1) << nout))
    return fail(ctx, OWQS_E_INVALID_ARG, "output must hold 2^(outputs) amplitudes");
  if (ctx->device < 0) return fail(ctx, OWQS_E_STATE, "host-only context (device -1) cannot run patterns");
  if (!ctx->noalloc) return fail(ctx, OWQS_E_STATE, "the allocation-free array was not resolved on this device");
  const bool lds = p->exec == OWQS_EXEC_AUTO && p->plan_width <= kLdsMaxWidth;
  if (p->dirty || (lds ? !p->dev_steps_valid : (!p->dev_fuse_valid || p->fuse_patched)))
    return fail(ctx, OWQS_E_STATE,
                "the plan is not on the device: run the pattern once with owqs_run after its last change");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ctx->noalloc);
  DevBook bk{};
  bk.sigma = reinterpret_cast<double *>(base + kOffSigma);
  bk.err = err ? err : reinterpret_cast<int *>(base + kOffErr);
  bk.partials = reinterpret_cast<double *>(base + kOffPartials);
  bk.probs = probs ? probs : reinterpret_cast<double *>(base + kOffProbs);
  float2 *psi = reinterpret_cast<float2 *>(base + kOffPsi);
  const int reduce = reduce_of(p);
  const bool empty_input = nin == 0 && input == nullptr;
  // sigma = 1 and the error word cleared (the previous call's values stay in
  // the array); the empty product state as psi[0] = 1
  e = launch_init(psi, bk, s, empty_input ? 1 : 0);
  if (e != hipSuccess) return hip_fail(ctx, e, "init");
  if (lds) {
    // whole pattern in one workgroup's LDS, straight from the caller's input
    // to the caller's output
    LdsItem proto = lds_proto(p);
    proto.in = static_cast<const float2 *>(input);
    proto.out = static_cast<float2 *>(output);
    proto.probs = bk.probs;
    proto.err = bk.err;
    e = launch_lds_shared(proto, 1, p->plan_width, reduce, 0, 0, size_t(p->n_meas), s);
    if (e != hipSuccess) return hip_fail(ctx, e, "LDS run");
    return OWQS_OK;
  }
  if (!empty_input) {
    e = hipMemcpyAsync(psi, input, n_in_amps * sizeof(float2), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "input copy");
  }
  e = launch_range(p, p->xsteps, 0, p->xsteps.size(), reduce, s, nullptr, nullptr, nullptr, psi, &bk);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  e = launch_read(psi, static_cast<float2 *>(output), int(nout), p->final_where.data(), p->final_factor,
                  reduce == kReduceRenorm ? bk.sigma : nullptr, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "read");
  return OWQS_OK;
}
