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

constexpr int kMaxPartials = 1 << 17;
// OWQS: windows with p = 1/2 exactly (an odd E(v, w) count) recorded in a row
// without summing the state; the next one sums and renormalises.
constexpr int kHalfRun = 128;
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
  const float2 *coef_dev;  // non-null: read the coefficient from device memory instead (drawn outcomes)
  const int *fold_dev;     // non-null (windows): swap, neg0, neg1 of the folded corrections from device memory
  double host_factor;   // (1/sqrt 2)^(N commands since the previous M)
  int reduce;           // ReduceMode
  int m_index;          // index of this M (probs slot)
  int prob_half;        // windows: p = 1/2 exactly (odd E(v, w) count); with kReduceNone, probs[m_index] = 1/2
  DevBook book;
};

// Shape of a window  N w; E...; M v; (X|Z on w)*  executed as one 2x2 update
// of v's slot (w takes that slot).  With a = psi[v = 0], b = psi[v = 1] at the
// index j of the other slots:
//   o0 = f (a + c sb b),  o1 = so1 f (a + s c sb b),
// sb = (-1)^parity(j & mask_b) (the E(v, x) with x != w), so1 =
// (-1)^parity(j & mask_o1) (the E(w, y) with y != v), s = -1 when E(v, w)
// occurs an odd number of times; then the folded corrections: swap (o0, o1)
// if `swap`, negate o0 / o1 if neg0 / neg1.
struct Window {
  uint64_t mask_b;
  uint64_t mask_o1;
  int swap, neg0, neg1;
  int vw_even;  // 1: E(v, w) occurs an even number of times (s = +1)
};

// One compiled step in device memory, for the kernels that walk a command
// table themselves (whole pattern resident in LDS).  24 bytes.
struct DevStep {
  uint8_t kind, n, b0, b1;  // step kind, live width before it, slots
  int32_t m_index;          // M / window: index of the measurement
  float2 coef;              // M / window: (-1)^o e^{-i theta}
  float host_factor;        // M / window: (1/sqrt 2)^(pending N)
  uint32_t pp;              // window: bit 0 swap, bit 1 negate 0, bit 2 negate 1, bit 3 vw_even,
                            // bit 4 sum its probability even when p = 1/2 exactly
  uint64_t mask_b;          // window: see Window
  uint64_t mask_o1;
};  // 40 bytes

__host__ __device__ inline Window window_of(const DevStep &st) {
  Window w{};
  w.mask_b = st.mask_b;
  w.mask_o1 = st.mask_o1;
  w.swap = int(st.pp & 1u);
  w.neg0 = int((st.pp >> 1) & 1u);
  w.neg1 = int((st.pp >> 2) & 1u);
  w.vw_even = int((st.pp >> 3) & 1u);
  return w;
}

// DK_U: windows in a row on one register-round position composed into one
// 2x2 map (see merge_round_windows); it takes a window's place in a sweep.
enum DevKind : uint8_t { DK_N = 0, DK_E = 1, DK_M = 2, DK_X = 3, DK_Z = 4, DK_J = 5, DK_R = 6, DK_S = 7, DK_U = 8 };

// ---- tile fusion (owqs_tile.hip)
constexpr int kLowBits = 5;            // slots 0..4 are always in a tile (256-byte runs)
constexpr int kMaxTileBits = 13;       // 2^13 complex64 = 64 KiB of LDS
constexpr int kDefaultTileBits = 12;   // 32 KiB tiles: four workgroups per CU
constexpr int kMinTileBits = 10;       // smallest tile the kernels take
constexpr int kTileMinWidth = 15;      // at least 2^5 tiles of 2^10; narrower runs stay one kernel per step
constexpr int kMaxGroupWindows = 32;
// A group that runs without a reduction (OWQS windows with p = 1/2 exactly)
// may hold more windows: the per-window sums only serve groups that reduce.
constexpr int kMaxHalfWindows = 128;
constexpr unsigned kTileGridCap = 4096;  // kMaxGroupWindows * kTileGridCap <= kMaxPartials
// Threads of a tile pass over 2^k-amplitude tiles, and the bits of the
// register cube each thread holds in a round (2^k / threads amplitudes).
constexpr int tile_threads(int tile_bits) { return tile_bits >= 13 ? 512 : tile_bits <= 11 ? 128 : 256; }
constexpr int tile_cube_bits(int tile_bits) {
  return tile_bits - (tile_bits >= 13 ? 9 : tile_bits <= 11 ? 7 : 8);
}

// One command of a fused group, with its slots mapped into the tile.
struct FuseOp {
  uint8_t kind;      // DK_J, DK_X, DK_E, DK_Z; DK_R, DK_S: round and sweep headers (see k_tile)
  uint8_t lb;        // J, X: local (tile) bit of the mixing slot
  uint8_t flags;     // J: bit 0 swap, 1 negate o0, 2 negate o1, 3 vw_even, 4 apply sigma;
                     // S: bit p set: the sweep has a window on cube position p
  uint8_t widx;      // J: index of the window inside its group
  int32_t m_index;   // J: measurement index; R: entries of the round (they follow it); S: its E / Z
  float2 coef;       // J: the factor f times the coefficient
  float f;           // J: host factor
  uint32_t lmask_b;  // J: local bits of mask_b;  E/Z: local bits that must all be 1;
                     // R: the cube's local bits, one per byte, ascending
  uint32_t lmask_o1; // J: local bits of mask_o1
  uint32_t rw_rs;    // J: sign bit of r (round_words)
  uint64_t omask_b;  // J: outer bits of mask_b;  E/Z: outer bits that must all be 1
  uint64_t omask_o1; // J: outer bits of mask_o1
  // J, for register rounds (round_words): fa, r fb and the sign of c0 as words
  // on a tile where the outer bits of both masks have even parity, and the
  // sign mask (0 or bit 31) of the folded exchange
  uint32_t rw_fa, rw_fbr, rw_cs, rw_fold;
};  // 64 bytes
// A DK_U row (a composed 2x2 map o0 = m00 a + m01 b, o1 = m10 a + m11 b on
// true amplitudes) keeps lb and holds its four complex entries as FP32 words:
// m00 in coef, m01 in (lmask_o1, rw_rs), m10 in (rw_fa, rw_fbr), m11 in
// (rw_cs, rw_fold); lmask_b, omask_b and omask_o1 are 0.

// A window's parameters with its tile-independent signs resolved, as a
// register round takes them: the window maps the pair (a, b) to
// o0 = fa a + t, o1 = fb a + r t with t = fa c0 b, the outputs exchanged by a
// folded X correction (flag bit 0).  Flag bits 1 and 2 negate o0 and o1;
// without flag bit 3, s1 = -1 (r = s1 fb / fa).  A window without local
// masks takes the exchange into its parameters (fa and fb exchanged, c0 ->
// r c0).  On a tile where the outer bits of mask_o1 have odd parity, fb and
// r change sign: with the exchange folded in, so do fa, r fb and c0, which is
// what rw_fold masks; an odd parity of mask_b's outer bits negates c0.
// Called wherever a window's flags, factor or coefficient are written (the
// plan compiler, and the kernel that resolves drawn outcomes).
__host__ __device__ inline void round_words(FuseOp &op) {
  const uint32_t kS = 0x80000000u, fl = op.flags;
  const bool sw = fl & 1u;
  const uint32_t n0 = (fl & 2u) ? kS : 0u, n1 = (fl & 4u) ? kS : 0u;
  const uint32_t sa = sw ? n1 : n0, sb = sw ? n0 : n1;
  const uint32_t rs = ((fl & 8u) ? 0u : kS) ^ sa ^ sb;
  uint32_t f;
  __builtin_memcpy(&f, &op.f, sizeof(f));
  uint32_t fa = f ^ sa, fb = f ^ sb, cs = sa;
  const bool fold = sw && (op.lmask_b | op.lmask_o1) == 0;
  if (fold) {
    const uint32_t t = fa;
    fa = fb;
    fb = t;
    cs ^= rs;
  }
  op.rw_fa = fa;
  op.rw_fbr = fb ^ rs;
  op.rw_cs = cs;
  op.rw_rs = rs;
  op.rw_fold = fold ? kS : 0u;
}

// A window's map on true amplitudes as a register round applies it (no
// masks, no sign pending on its position): t = c b, o0 = fa a + t, and the
// round stores fbr a + t for o1 = r (fbr a + t), r the sign of rw_rs; so
// [[fa, c], [r fbr, r c]], row-major, as (re, im) pairs.  From the round
// words (round_words), on the host (plan compiler) and on the device (drawn
// outcomes).
__host__ __device__ inline void window_map(const FuseOp &w, double m[8]) {
  const uint32_t cs = w.rw_cs & 0x80000000u;
  uint32_t cx, cy;
  __builtin_memcpy(&cx, &w.coef.x, sizeof(cx));
  __builtin_memcpy(&cy, &w.coef.y, sizeof(cy));
  cx ^= cs;
  cy ^= cs;
  float fcx, fcy, fa, fbr;
  __builtin_memcpy(&fcx, &cx, sizeof(fcx));
  __builtin_memcpy(&fcy, &cy, sizeof(fcy));
  __builtin_memcpy(&fa, &w.rw_fa, sizeof(fa));
  __builtin_memcpy(&fbr, &w.rw_fbr, sizeof(fbr));
  const double r = (w.rw_rs & 0x80000000u) ? -1.0 : 1.0;
  m[0] = fa;
  m[1] = 0.0;
  m[2] = fcx;
  m[3] = fcy;
  m[4] = r * fbr;
  m[5] = 0.0;
  m[6] = r * fcx;
  m[7] = r * fcy;
}

// u <- w u for 2x2 complex maps (row-major, (re, im) pairs), in FP64.
__host__ __device__ inline void map_left(const double w[8], double u[8]) {
  double n[8];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double ar = w[4 * i], ai = w[4 * i + 1], br = w[4 * i + 2], bi = w[4 * i + 3];
      const double cr = u[2 * j], ci = u[2 * j + 1], dr = u[4 + 2 * j], di = u[4 + 2 * j + 1];
      n[4 * i + 2 * j] = ar * cr - ai * ci + br * dr - bi * di;
      n[4 * i + 2 * j + 1] = ar * ci + ai * cr + br * di + bi * dr;
    }
  for (int k = 0; k < 8; ++k) u[k] = n[k];
}

// The entries of a composed map (DK_U row), each rounded once to FP32.
__host__ __device__ inline void map_store(FuseOp &row, const double u[8]) {
  float f[8];
  for (int k = 0; k < 8; ++k) f[k] = float(u[k]);
  row.coef = make_float2(f[0], f[1]);
  __builtin_memcpy(&row.lmask_o1, &f[2], 4);
  __builtin_memcpy(&row.rw_rs, &f[3], 4);
  __builtin_memcpy(&row.rw_fa, &f[4], 4);
  __builtin_memcpy(&row.rw_fbr, &f[5], 4);
  __builtin_memcpy(&row.rw_cs, &f[6], 4);
  __builtin_memcpy(&row.rw_fold, &f[7], 4);
}

struct TileArgs {
  uint64_t tmask;    // global slots in the tile (tile bit i = the i-th lowest)
  uint64_t omask;    // the other live slots (outer bit i = the i-th lowest)
  // several vectors (sets) at once: set y at psi + y * set_stride, window
  // coefficients coefs[m_index * nsets + y] (coefs null: one vector, the
  // coefficients of the command table)
  uint64_t set_stride;
  const float2 *coefs;
  // non-null: the folded corrections of window m are folds[3 m .. 3 m + 2] =
  // {swap, neg0, neg1} (resolved per run from drawn outcomes)
  const int *folds;
  // non-null: every window of the group has p = 1/2 exactly (an odd E(v, w)
  // count) and the pass runs without a reduction; workgroup (0, 0) writes
  // book.probs[half_m[i]] = 1/2 for its nwin windows
  const int *half_m;
  int nsets;
  int n, k, nops, nwin;
  int runs;          // 1: some consecutive unmasked windows run in registers (see k_tile)
  // 1 (set per launch): the pass sums the squared norm of its output into
  // partials (k_tile: one per block; k_tile_multi: one per tile), from which
  // k_finish_renorm / k_finish_multi reset sigma
  int renorm;
  // 1 (set per launch): every window slot of the group's rounds holds a
  // composed map (DK_U) and the pass sums no window: the kernel variant with
  // only the map path runs (one code path per position keeps the amplitudes
  // in their registers)
  int maps;
  uint8_t tpos[16];  // global slot of tile bit i (tpos[i] = i for i < kLowBits)
  uint8_t opos[48];  // global slots of the bits outside the tile, ascending (n - k of them)
};

// One pattern's tile group inside a multi-pattern tile launch (batched runs):
// the launch covers the tiles of every entry, entry e owning global tiles
// first_tile .. first_tile + 2^(ta.n - ta.k) - 1.
struct MultiTile {
  float2 *psi;            // the pattern's live vector
  const FuseOp *ops;      // the group's commands
  double *partials;       // reduce: window w of tile t at partials[w * ntiles + t]
  const double *sigma;    // the pattern's FP64 scale (read when reduce == kReduceRenorm)
  double *probs;          // the pattern's probabilities (ta.half_m: 1/2 written by tile 0)
  TileArgs ta;
  int reduce;             // ReduceMode of this group (kReduceNone for groups of p = 1/2 windows)
  uint32_t first_tile;
};

// One pattern's group finish inside a multi-pattern finishing launch.
struct MultiFinish {
  DevBook book;
  const int *m_of_window;  // measurement index of each window of the group
  int nwin;
  int reduce;
  uint32_t ntiles;         // partials per window
  int renorm;              // 1: the group's output norm resets sigma (nwin = 1, one partial per tile)
};

// Start and read-out of one pattern of a batched run.
struct BatchIo {
  float2 *psi;             // live vector
  const float2 *in;        // 2^nin input amplitudes, or null (empty product state)
  float2 *out;             // 2^nout output amplitudes
  DevBook book;
  double final_factor;
  int nin, nout, reduce;
  int where[kWhereMax];    // slot of output k
};

// One pattern of an LDS-resident batch.
struct LdsItem {
  const DevStep *steps;
  const float2 *in;     // 2^nin amplitudes (ignored for basis inputs)
  float2 *out;          // 2^nout amplitudes
  double *probs;        // n_meas entries, or null
  int *err;             // {first failing M (or item), kind}: this item's error slot
  double final_factor;
  int nsteps, nin, nout, basis;  // basis >= 0: input is |basis>
  int reduce;                    // ReduceMode of this item (k_lds_batch)
  int where[kWhereMax];
};

constexpr int kLdsMaxWidth = 14;  // 2^14 complex64 = 128 KiB of the 160 KiB LDS

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
hipError_t launch_jwindow(float2 *psi, int n, int b, const MeasureArgs &a, const Window &win, hipStream_t s,
                          unsigned *grid);
hipError_t launch_finish(const MeasureArgs &a, unsigned nparts, hipStream_t s);
hipError_t launch_read(const float2 *psi, float2 *out, int nout, const int *where, double host_factor,
                       const double *sigma, hipStream_t s);


// ---- owqs_batch.hip
// Run `count` items, each a whole pattern resident in the LDS of one
// workgroup (live width <= kLdsMaxWidth).  `width` is the largest live width
// of any item (sets the dynamic LDS size).  Errors (zero probability, failed
// determinism check) go to each item's err slot: err[0] = first failing M.
hipError_t launch_lds_batch(const LdsItem *items, int count, int width, hipStream_t s);
// Raise k_lds_batch's dynamic LDS limit to 2^kLdsMaxWidth amplitudes (once,
// outside any graph capture).
hipError_t lds_batch_prepare();
// Batched runs: start every wide pattern (sigma, error word, input into its
// live vector) and read every output (gather and scale), one launch each.
hipError_t launch_batch_start(const BatchIo *ios, int count, int max_nin, hipStream_t s);
hipError_t launch_batch_read(const BatchIo *ios, int count, int max_nout, hipStream_t s);
// Tile groups of many patterns in one launch (entries sorted by first_tile,
// all with tile bits k, the same `runs` and, as `red`, all with or all
// without the FP64 window sums; `maps`: every entry's rounds hold composed
// maps only, ta.maps), and their group finishes.
hipError_t launch_tile_multi(const MultiTile *ents, int nent, uint32_t total, int k, bool runs, bool red,
                             bool maps, hipStream_t s);
hipError_t launch_finish_multi(const MultiFinish *fins, int nfin, int maxwin, hipStream_t s);
// Items share one command table and differ only by input: item k runs on
// basis state |first + k> (basis_mode = 1) or on in + k * 2^nin, and writes
// out + k * 2^nout.  Errors go to proto.err with err[0] = first failing item.
hipError_t launch_lds_shared(const LdsItem &proto, int count, int width, int reduce, uint32_t first,
                             int basis_mode, size_t probs_stride, hipStream_t s);


// ---- owqs_adjoint.hip: B sets side by side, set = blockIdx.y, set stride
// `stride` amplitudes.  Steps are DevStep rows (N, E, X, Z, J); J reads its
// per-set coefficient from coefs[set].
hipError_t launch_b_init(float2 *psi, size_t stride, int nsets, int nin, const float2 *in, hipStream_t s);
hipError_t launch_b_step(const DevStep &st, float2 *psi, size_t stride, int nsets, const float2 *coefs,
                         hipStream_t s);
unsigned adj_blocks(int n);   // blocks per set of launch_b_window_adj at width n
hipError_t launch_b_window_adj(const DevStep &st, const float2 *psi_in, float2 *lam, size_t stride, int nsets,
                               const float2 *coefs, double *partials, hipStream_t s);
hipError_t launch_b_window_rev(const DevStep &st, float2 *psi, float2 *lam, size_t stride, int nsets,
                               const float2 *coefs, double *partials, unsigned prow, hipStream_t s);
unsigned loss_blocks(int n);  // blocks per set of launch_b_loss at width n
hipError_t launch_b_loss(const float2 *psi, float2 *lam, size_t stride, int nsets, int n, const int *obs_bits,
                         int nobs, double ff2, double *partials, hipStream_t s);
hipError_t launch_b_reduce(const double *partials, int nq, int nsets, int nblk, const int *out_col,
                           const double *scale, double *out, size_t out_stride, hipStream_t s);


// ---- owqs_tile.hip: one group of commands in one pass; *grid receives the
// block count, which launch_finish_group needs to reduce the partials.
hipError_t launch_tile(float2 *psi, const TileArgs &ta, const FuseOp *ops, const MeasureArgs &a, hipStream_t s,
                       unsigned *grid);
// sigma = 1 / sqrt(sum of partials[0 .. nblk)) after a pass with TileArgs::renorm.
hipError_t launch_finish_renorm(const DevBook &book, unsigned nblk, hipStream_t s);
hipError_t launch_finish_group(const MeasureArgs &a, const int *m_of_window, int nwin, unsigned nblk,
                               hipStream_t s);
// Raise k_tile's dynamic LDS limit to 64 KiB; call outside stream capture.
hipError_t tile_prepare();

// The group on `nsets` vectors at once (EOWQS scale, no probabilities).
hipError_t launch_tile_sets(float2 *psi, const TileArgs &ta, const FuseOp *ops, int nsets, size_t set_stride,
                            const float2 *coefs, hipStream_t s);
// Reverse sweep of the group on nsets (psi, lam) pairs: psi goes from the
// group's output back to its input, lam (the adjoint state) from after the
// group to before it, and partials[((q_first + g) * nsets + y) * nblk + block]
// receives this block's gradient sum of window g (windows must be invertible).
hipError_t launch_tile_rev(float2 *psi, float2 *lam, const TileArgs &ta, const FuseOp *ops, int nsets,
                           size_t set_stride, const float2 *coefs, double *partials, int q_first, unsigned nblk,
                           hipStream_t s);
unsigned tile_grid(const TileArgs &ta);

// ---- drawn outcomes (owqs_sample.hip)
constexpr unsigned kSampleGrid = 4096;  // 2 * kSampleGrid <= kMaxPartials
// Signals of a command: XOR of the drawn outcomes outc[dom[off .. off+len)].
struct SigRef {
  int off, len;
};
// X (x = 1) or Z (x = 0) on slot b at live width n when its signal is 1.
hipError_t launch_s_pauli(float2 *psi, int n, int b, int x, SigRef sig, const int *dom, const int *outc,
                          hipStream_t s);
// Probability pass of M at slot b: per-block FP64 sums of |psi_0 + c0 psi_1|^2
// (c0 = e^{-i theta}, theta from alpha and the s, t signals, Eq. 2) into
// partials[0 .. grid) and of |psi_0|^2 + |psi_1|^2 into partials[kSampleGrid ..)
// (grid <= kSampleGrid).
hipError_t launch_s_prob(const float2 *psi, int n, int b, double alpha, SigRef sg, SigRef tg, const int *dom,
                         const int *outc, double *partials, unsigned *grid, hipStream_t s);
// One block: p_0 from the partials, outcome o = (u[m] <= p_0 ? 0 : 1) into
// outc[m] and the collapse coefficient (-1)^o e^{-i theta} into *coef.
hipError_t launch_s_decide(const double *partials, unsigned nparts, const double *u, int m, double alpha,
                           SigRef sg, SigRef tg, const int *dom, int *outc, float2 *coef, hipStream_t s);
// A correction folded into a drawn window: X (x = 1) or Z on the new qubit w
// when the signal sig is 1.
struct FoldRef {
  int x;
  SigRef sig;
};
// A drawn window of a plan whose every M is such a window (p = 1/2 for every
// state): its outcome is u[m] <= 1/2, known before the run, like every
// outcome its signals read.
struct DrawWin {
  double alpha;
  SigRef s, t;
  int m, fold_off, fold_len;
  int fop;  // the window's row in the pattern's tile-pass command table, or -1
};
// All drawn windows at once, one thread each: outc[m], the collapse
// coefficient ctab[m] and the folded corrections ftab[3 m .. 3 m + 2] (swap,
// negate o0, negate o1), every signal taken from the uniforms directly; a
// window inside a tile pass also gets them in its command row (fops[fop]:
// coef and flag bits 0-2), so that the pass runs like a forced one.
// Composed maps of a drawn run from the rows k_s_resolve wrote: map i's
// entry starts at refs[off[i]] (its row in mrows, its window count, its
// windows' rows in fops).
hipError_t launch_s_compose(const FuseOp *fops, FuseOp *mrows, const int *refs, const int *off, int nmaps,
                            hipStream_t s);
hipError_t launch_s_resolve(const DrawWin *wins, int nwin, const double *u, const int *dom, const FoldRef *folds,
                            int *outc, float2 *ctab, int *ftab, FuseOp *fops, hipStream_t s);
// One thread, for a window whose E count between v and w is odd (outcome
// probability exactly 1/2, Sec. 4.5): o = (u[m] <= 1/2 ? 0 : 1) into outc[m],
// the coefficient into *coef, then the folded corrections folds[0 .. nf)
// resolved with the drawn outcomes into fold[0..2] = {swap, neg0, neg1}.
hipError_t launch_s_jdecide(const double *u, int m, double alpha, SigRef sg, SigRef tg, const int *dom, int *outc,
                            float2 *coef, const FoldRef *folds, int nf, int *fold, hipStream_t s);


// ---- sub-state executor (owqs_substate.hip)
constexpr int kMaxFactors = kWhereMax;  // factors of a read-out (each holds >= 1 output)
// Read-out of a product state: factor f was read into stage[off[f] ..) with
// its qubits in output order and owns the output bits mask[f]; the scalar
// (product of the fully measured sub-states) is stage[scalar_off].
struct AssembleArgs {
  uint64_t off[kMaxFactors];
  uint64_t mask[kMaxFactors];
  uint64_t scalar_off;
  int nf;
};
// sigma[0 .. nchains) = 1 and the error word cleared.
hipError_t launch_sub_start(double *sigma, int nchains, int *err, hipStream_t s);
// psi[0] = 1 (a sub-state with no qubit yet).
hipError_t launch_sub_init(float2 *psi, hipStream_t s);
// In place: base (2^a amplitudes, capacity 2^(a+b)) becomes base (x) top,
// base's qubits on the low a bits; *sig_a *= *sig_b.  a, b >= 1.
hipError_t launch_kron(float2 *base, int a, const float2 *top, int b, double *sig_a, const double *sig_b,
                       hipStream_t s);
// v[0] = v[0] v[1] ... v[count - 1] (count may be 0: v[0] = 1).
hipError_t launch_cprod(float2 *v, int count, hipStream_t s);
hipError_t launch_assemble(float2 *out, int nout, const float2 *stage, const AssembleArgs &a, hipStream_t s);

}  // namespace owqs
