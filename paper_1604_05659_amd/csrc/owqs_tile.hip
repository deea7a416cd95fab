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
// kernel chains p_g = n_g / (2 n_{g-1}) (n_0 = 1: a group with windows
// scales its tile by sigma as it loads it) and sets sigma = 1 / sqrt(n_last).  A group whose
// windows all have p = 1/2 exactly (an odd E(v, w) count) runs without the
// sums when the host says so (TileArgs::half_m): it records p = 1/2, keeps
// the norm of its input, and leaves sigma as it is.
#include <type_traits>

#include "owqs_internal.h"

namespace owqs {
namespace {

constexpr int kTT = 256;  // threads per workgroup of the finishing kernel

// Threads per workgroup of a tile pass (tile_threads): 512 (8 waves) for
// 2^13-amplitude tiles, so that a CU holding two such tiles still runs 16
// waves; 128 for 2^10 and 2^11 tiles, so that every thread has 8 or 16
// amplitudes to work on per command (the per-command decoding is paid once
// per wave).
constexpr int log2_threads(int t) { return t == 512 ? 9 : t == 256 ? 8 : 7; }

__device__ __forceinline__ uint32_t ins0u(uint32_t x, int b) { return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1)); }
__device__ __forceinline__ uint32_t par64(uint64_t x) { return uint32_t(__popcll(x) & 1); }
__device__ __forceinline__ uint32_t par32(uint32_t x) { return uint32_t(__popc(x) & 1); }
__device__ __forceinline__ float xsign(float x, uint32_t s) { return __uint_as_float(__float_as_uint(x) ^ s); }
__device__ __forceinline__ float2 xsign2(float2 v, uint32_t s) { return make_float2(xsign(v.x, s), xsign(v.y, s)); }
// |a|^2 + |b|^2 of one pair: four FP32 products summed in FP32 (relative
// error below 3 ulp), returned as FP64, so that a thread's, a wave's, a
// workgroup's and the tiles' sums over pairs accumulate in FP64 and the
// error stays that of one pair sum however many pairs there are
__device__ __forceinline__ double nrm2d(float2 a, float2 b) {
  return double(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
}
// An empty asm statement that the compiler must assume changes x: values
// computed from x before it are not reused after it (no instructions).
__device__ __forceinline__ void opaque(uint64_t &x) {
  uint32_t lo = uint32_t(x), hi = uint32_t(x >> 32);
  asm volatile("" : "+v"(lo), "+v"(hi));
  x = (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ void opaque32(uint32_t &x) { asm volatile("" : "+v"(x)); }
// x in a vector register (an empty asm statement that takes it as one).
__device__ __forceinline__ float in_vgpr(float x) {
  asm volatile("" : "+v"(x));
  return x;
}
// The vector as a buffer resource, for live widths up to 28 (byte offsets
// below 2^31): a load or store then takes the uniform part of its offset in
// a scalar register and the thread's part in a vector one, with no vector
// instruction to form the address.  The record count, 2^32 - 1 bytes at
// most, leaves the last dword of a 2^29-amplitude vector outside the range
// (read as 0, not written), so width 29 takes the global path.  Word 3 is
// the format CDNA's untyped buffer access takes (32-bit data).
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(float2 *psi) {
  return __builtin_amdgcn_make_buffer_rsrc(psi, 0, 0xFFFFFFFF, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(w[0]), __uint_as_float(w[1]));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float2 v) {
  const u32x2 w = {__float_as_uint(v.x), __float_as_uint(v.y)};
  __builtin_amdgcn_raw_buffer_store_b64(w, r, voff, soff, 0);
}
__device__ __forceinline__ float2 &at(char *lds, uint32_t byte_off) { return *reinterpret_cast<float2 *>(lds + byte_off); }

// One command of the group, read as whole dwords from a uniform address so
// that it comes through scalar loads (its byte fields are unpacked after).
__device__ __forceinline__ FuseOp load_op(const FuseOp *__restrict__ ops, int o) {
  static_assert(sizeof(FuseOp) == 64, "FuseOp is 16 dwords");
  // the command table is never written by the kernels: read it through the
  // constant address space, which the scalar unit may always load
  typedef const __attribute__((address_space(4))) uint32_t cword;
  cword *src = reinterpret_cast<cword *>(reinterpret_cast<uintptr_t>(ops)) + 16 * __builtin_amdgcn_readfirstlane(o);
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = src[i];
  FuseOp op;
  __builtin_memcpy(&op, w, sizeof(op));
  return op;
}

// x plus the FP64 value of another lane chosen by a DPP control (two 32-bit
// DPP moves); lanes whose source is outside the row mask or the row add 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double add_dpp(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(u), kCtrl, kRowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(u >> 32), kCtrl, kRowMask, 0xf, false);
  return x + __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Sum of x over the 64 lanes of the wave, valid in lane 63: shifts by 1, 2,
// 4 and 8 inside each 16-lane row leave the row sums in lanes 15, 31, 47 and
// 63; the row broadcasts 15 and 31 then add them up into lane 63.
__device__ __forceinline__ double wave_sum_to_last(double x) {
  x = add_dpp<0x111, 0xf>(x);  // row_shr:1
  x = add_dpp<0x112, 0xf>(x);  // row_shr:2
  x = add_dpp<0x114, 0xf>(x);  // row_shr:4
  x = add_dpp<0x118, 0xf>(x);  // row_shr:8
  x = add_dpp<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = add_dpp<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Window coefficient of measurement m for set blockIdx.y (read-only table,
// uniform over the workgroup: scalar loads through the constant space).
__device__ __forceinline__ float2 set_coef(const TileArgs &ta, int m) {
  typedef const __attribute__((address_space(4))) float cf;
  cf *tab = reinterpret_cast<cf *>(reinterpret_cast<uintptr_t>(ta.coefs)) + 2 * (size_t(m) * ta.nsets + blockIdx.y);
  return make_float2(tab[0], tab[1]);
}

// A window's flags, with the folded corrections (bits 0-2) from the device
// table when they were resolved per run (drawn outcomes).
__device__ __forceinline__ uint32_t op_flags(const FuseOp &op, const TileArgs &ta) {
  uint32_t fl = op.flags;
  if (ta.folds) {
    typedef const __attribute__((address_space(4))) int ci;
    ci *t = reinterpret_cast<ci *>(reinterpret_cast<uintptr_t>(ta.folds)) + 3 * op.m_index;
    fl = (fl & ~7u) | (t[0] ? 1u : 0u) | (t[1] ? 2u : 0u) | (t[2] ? 4u : 0u);
  }
  return fl;
}

// Deposit the low bits of x, lowest first, into the set bits of mask.
__device__ __forceinline__ uint64_t pdep64(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bb = 1; mask; bb <<= 1) {
    const uint64_t low = mask & (~mask + 1);
    if (x & bb) r |= low;
    mask ^= low;
  }
  return r;
}

// Negate the tile elements whose local bits m are all set (E: two bits,
// Z: one; no bit when the factor depends on outer bits only).  Only the
// affected quarter / half / whole tile is visited: element
// ins0(ins0(q, lo), hi) | m for q < 2^(k-2), and so on.  Insertion of zero
// bits acts on each bit separately, so the part from the thread index and the
// part from the loop counter r (uniform) are combined with an OR.
template <int kTB, int kT>
__device__ __forceinline__ void diag_flip(char *lds, uint32_t tid, uint32_t m) {
  constexpr int kPer = (1 << kTB) / kT;
  constexpr uint32_t kNeg = 0x80000000u;
  const int nb = __popc(m);
  if (nb == 2) {
    const int lo = __ffs(m) - 1, hi = 31 - __clz(m);
    const uint32_t et = (ins0u(ins0u(tid, lo), hi) | m) << 3;
#pragma unroll
    for (int r = 0; r < kPer / 4; ++r) {
      const uint32_t a = et | (ins0u(ins0u(uint32_t(r) * kT, lo), hi) << 3);
      at(lds, a) = xsign2(at(lds, a), kNeg);
    }
  } else if (nb == 1) {
    const int lo = __ffs(m) - 1;
    const uint32_t et = (ins0u(tid, lo) | m) << 3;
#pragma unroll
    for (int r = 0; r < kPer / 2; ++r) {
      const uint32_t a = et | (ins0u(uint32_t(r) * kT, lo) << 3);
      at(lds, a) = xsign2(at(lds, a), kNeg);
    }
  } else {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const uint32_t a = (tid + uint32_t(r) * kT) << 3;
      at(lds, a) = xsign2(at(lds, a), kNeg);
    }
  }
}

// X: swap the element pairs that differ in local bit lb.
template <int kTB, int kT>
__device__ __forceinline__ void pair_swap(char *lds, uint32_t tid, int lb) {
  constexpr int kPairs = (1 << kTB) / kT / 2;
  const uint32_t et = ins0u(tid, lb) << 3, bit8 = 8u << lb;
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    const uint32_t a0 = et | (ins0u(uint32_t(r) * kT, lb) << 3), a1 = a0 | bit8;
    const float2 x = at(lds, a0);
    at(lds, a0) = at(lds, a1);
    at(lds, a1) = x;
  }
}

// How a window's pair update is compiled (WinP::kind).  A window maps the
// element pair (a, b) that differs in its local bit to
//   t = fc0 b,  o0 = fa a + t,  o1 = fb a + r t   (r = +-1),
// the outputs exchanged by a folded X correction.  Without local masks the
// exchange is folded into the parameters (o1 = fb a + r fc0 b in place of
// o0 is the same form with fa and fb exchanged and fc0 -> r fc0, r kept),
// and r is compiled in: kWinPlus, kWinMinus.  With local masks (b negated
// where the local bits lmb have odd parity, o1 where lmo has) the signs are
// applied at run time and the exchange is compiled in: kWinMasked,
// kWinMaskedSw.
enum : int { kWinPlus = 0, kWinMinus = 1, kWinMasked = 2, kWinMaskedSw = 3 };

// A window's per-tile parameters: the tile-constant signs and the folded
// corrections resolved into fa, fb, fc0 and the sign of t in o1.
struct WinP {
  float fa, fb;
  float2 fc0;
  uint32_t rsign, lmb, lmo;  // rsign: sign bit of r
  int lb, widx, kind;
};

// All of it is sign-bit work on uniform words (scalar instructions) except
// for runs with one coefficient per set: FuseOp::coef holds the window's
// factor times its coefficient, so fc0 = fa c0 is that product with a sign.
// Sigma, which the group's first window applies (flag bit 4), is applied to
// the tile as it is loaded (see tile_one).  A register round passes two more
// signs: cs, a sign of fc0 (the pending sign of the window's position), and
// fold_r, which makes fb carry r (the round stores r o1).  Every sign is
// applied to the words before they move to vector registers: a sign applied
// after the move would cost a vector instruction per word and window.
__device__ __forceinline__ WinP prep_window(const FuseOp &op, uint64_t ob, const TileArgs &ta, uint32_t cs = 0u,
                                            bool fold_r = false) {
  constexpr uint32_t kS = 0x80000000u;
  WinP w;
  if (!ta.coefs && !ta.folds) {
    // the words of the command table (round_words) hold every sign but those
    // of this tile: p1 and p2, the parities of the outer bits of mask_o1 and
    // mask_b (a dozen scalar instructions)
    const uint32_t p1 = par64(ob & op.omask_o1) << 31, p2 = par64(ob & op.omask_b) << 31;
    const uint32_t x = p1 & op.rw_fold;
    const uint32_t rs = op.rw_rs ^ p1, fbr = op.rw_fbr ^ x, c = op.rw_cs ^ x ^ p2 ^ cs;
    w.fa = in_vgpr(__uint_as_float(op.rw_fa ^ x));
    w.fb = in_vgpr(__uint_as_float(fold_r ? fbr : fbr ^ rs));
    w.fc0 = make_float2(in_vgpr(__uint_as_float(__float_as_uint(op.coef.x) ^ c)),
                        in_vgpr(__uint_as_float(__float_as_uint(op.coef.y) ^ c)));
    w.rsign = rs;
    w.lmb = op.lmask_b;
    w.lmo = op.lmask_o1;
    w.lb = op.lb;
    w.widx = op.widx;
    const bool masked = (op.lmask_b | op.lmask_o1) != 0;
    w.kind = masked ? ((op.flags & 1u) ? kWinMaskedSw : kWinMasked) : (rs ? kWinMinus : kWinPlus);
    return w;
  }
  // coefficients per set, or corrections read per run: every sign from the flags
  const uint32_t fl = op_flags(op, ta);
  const bool sw = fl & 1u;
  // signs of fa, fb (the factor) and of c0 (the coefficient) on this tile:
  // flag bits 1 and 2 negate o0 and o1, which are exchanged by the swap
  const uint32_t n0 = (fl << 30) & kS, n1 = (fl << 29) & kS;
  const uint32_t sa = sw ? n1 : n0;
  const uint32_t sb = (par64(ob & op.omask_o1) << 31) ^ (sw ? n0 : n1);
  const uint32_t sc = par64(ob & op.omask_b) << 31;
  uint32_t cx = __float_as_uint(op.coef.x), cy = __float_as_uint(op.coef.y);
  if (ta.coefs) {  // one coefficient per set: uniform, back to scalar words
    const float2 cw = set_coef(ta, op.m_index);
    cx = __builtin_amdgcn_readfirstlane(__float_as_uint(op.f * cw.x));
    cy = __builtin_amdgcn_readfirstlane(__float_as_uint(op.f * cw.y));
  }
  const uint32_t f = __float_as_uint(op.f);
  uint32_t fa = f ^ sa, fb = f ^ sb;
  uint32_t c0 = sa ^ sc ^ cs;  // the sign of fc0 = fa c0
  // o1 = fb a + fb s1 c0 b = fb a + r fc0 b, r = s1 fb / fa (|fa| = |fb|)
  const uint32_t rs = ((fl & 8u) ? 0u : kS) ^ sa ^ sb;  // sign bit of r
  const bool masked = (op.lmask_b | op.lmask_o1) != 0;
  if (!masked && sw) {
    const uint32_t t = fa;
    fa = fb;
    fb = t;
    c0 ^= rs;
  }
  if (fold_r) fb ^= rs;
  // the factors go to vector registers: the window arithmetic of the other
  // paths then takes the short (VOP2) encodings, which scalar operands rule out
  w.fa = in_vgpr(__uint_as_float(fa));
  w.fb = in_vgpr(__uint_as_float(fb));
  w.fc0 = make_float2(in_vgpr(__uint_as_float(cx ^ c0)), in_vgpr(__uint_as_float(cy ^ c0)));
  w.rsign = rs;
  w.lmb = op.lmask_b;
  w.lmo = op.lmask_o1;
  w.lb = op.lb;
  w.widx = op.widx;
  w.kind = masked ? (sw ? kWinMaskedSw : kWinMasked) : (rs ? kWinMinus : kWinPlus);
  return w;
}

// A window on one pair in registers: a at local index e0 (bit lb = 0), b at
// e0 with bit lb set.
template <int kKind>
__device__ __forceinline__ void win_apply(const WinP &w, uint32_t e0, float2 &a, float2 &b) {
  constexpr bool kMasked = kKind >= kWinMasked;
  float2 bb = b;
  float fbe = w.fb;
  uint32_t ts = w.rsign;
  if (kMasked) {
    bb = xsign2(bb, par32(e0 & w.lmb) << 31);
    const uint32_t so = par32(e0 & w.lmo) << 31;
    fbe = xsign(w.fb, so);
    ts ^= so;
  }
  const float2 t = make_float2(w.fc0.x * bb.x - w.fc0.y * bb.y, w.fc0.x * bb.y + w.fc0.y * bb.x);
  const float2 p0 = make_float2(fmaf(w.fa, a.x, t.x), fmaf(w.fa, a.y, t.y));
  float2 p1;
  if (kKind == kWinPlus) {
    p1 = make_float2(fmaf(w.fb, a.x, t.x), fmaf(w.fb, a.y, t.y));
  } else if (kKind == kWinMinus) {
    p1 = make_float2(fmaf(w.fb, a.x, -t.x), fmaf(w.fb, a.y, -t.y));
  } else {
    const float2 te = xsign2(t, ts);
    p1 = make_float2(fmaf(fbe, a.x, te.x), fmaf(fbe, a.y, te.y));
  }
  constexpr bool kSw = kKind == kWinMaskedSw;
  a = kSw ? p1 : p0;
  b = kSw ? p0 : p1;
}

// One window over the tile: every element pair that differs in local bit
// lb.  Returns this thread's sum of |o0|^2 + |o1|^2 in FP64 (kAcc).
template <int kKind, bool kAcc, int kTB, int kT>
__device__ __forceinline__ double window_pass(char *lds, uint32_t tid, const WinP &w) {
  constexpr int kPairs = (1 << kTB) / kT / 2;
  const uint32_t et = ins0u(tid, w.lb), bit8 = 8u << w.lb;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    const uint32_t e0 = et | ins0u(uint32_t(r) * kT, w.lb);
    const uint32_t a0 = e0 << 3, a1 = a0 | bit8;
    float2 a = at(lds, a0), b = at(lds, a1);
    win_apply<kKind>(w, e0, a, b);
    at(lds, a0) = a;
    at(lds, a1) = b;
    if (kAcc) acc += nrm2d(a, b);
  }
  return acc;
}

// The unmasked window with a mixing bit below the thread index bits: pair r
// of the thread is then at a fixed offset from the thread's first pair.
template <int kKind, bool kAcc, int kTB, int kT>
__device__ __forceinline__ double window_low(char *lds, uint32_t tid, const WinP &w) {
  static_assert(kKind == kWinPlus || kKind == kWinMinus, "unmasked windows only");
  constexpr int kPairs = (1 << kTB) / kT / 2;
  constexpr int kLogT = log2_threads(kT);
  const uint32_t a0t = ins0u(tid, w.lb) << 3, a1t = a0t | (8u << w.lb);
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    // pair index tid + r kT with lb < log2 kT: insertion shifts r kT up by one
    const uint32_t off = uint32_t(r) << (kLogT + 4);
    float2 a = at(lds, a0t + off), b = at(lds, a1t + off);
    win_apply<kKind>(w, 0u, a, b);
    at(lds, a0t + off) = a;
    at(lds, a1t + off) = b;
    if (kAcc) acc += nrm2d(a, b);
  }
  return acc;
}

template <bool kAcc, int kTB, int kT>
__device__ __forceinline__ double window_single(char *lds, uint32_t tid, const WinP &w) {
  constexpr int kLogT = log2_threads(kT);
  switch (w.kind) {
    case kWinMasked: return window_pass<kWinMasked, kAcc, kTB, kT>(lds, tid, w);
    case kWinMaskedSw: return window_pass<kWinMaskedSw, kAcc, kTB, kT>(lds, tid, w);
    case kWinMinus:
      return w.lb < kLogT ? window_low<kWinMinus, kAcc, kTB, kT>(lds, tid, w)
                          : window_pass<kWinMinus, kAcc, kTB, kT>(lds, tid, w);
    default:
      return w.lb < kLogT ? window_low<kWinPlus, kAcc, kTB, kT>(lds, tid, w)
                          : window_pass<kWinPlus, kAcc, kTB, kT>(lds, tid, w);
  }
}

__device__ __forceinline__ double nrm4(float2 a, float2 b, float2 c, float2 d) {
  return nrm2d(a, b) + nrm2d(c, d);
}

// Two consecutive windows A, B on different local bits in one LDS pass:
// each thread takes quads of elements (all values of the two bits), applies
// A to its two pairs, then B to its two pairs, in registers.  Half the LDS
// traffic and barriers of two passes.
template <bool kAcc, int kKA, int kKB, bool kMid, int kTB, int kT>
__device__ __forceinline__ void window_pair(char *lds, uint32_t tid, const WinP &A, const WinP &B, uint32_t mid,
                                            double &acc_a, double &acc_b) {
  constexpr int kQuads = (1 << kTB) / kT / 4;
  const int lo = A.lb < B.lb ? A.lb : B.lb, hi = A.lb < B.lb ? B.lb : A.lb;
  const uint32_t ba = 8u << A.lb, bb = 8u << B.lb;
#pragma unroll
  for (int r = 0; r < kQuads; ++r) {
    const uint32_t el = ins0u(ins0u(tid + uint32_t(r) * kT, lo), hi), e = el << 3;
    float2 x00 = at(lds, e), x10 = at(lds, e | ba), x01 = at(lds, e | bb), x11 = at(lds, e | ba | bb);
    win_apply<kKA>(A, el, x00, x10);
    win_apply<kKA>(A, el | (bb >> 3), x01, x11);
    if (kAcc) acc_a += nrm4(x00, x10, x01, x11);
    if (kMid) {  // an E / Z between the windows: negate where its local bits are all set
      if ((el & mid) == mid) x00 = xsign2(x00, 0x80000000u);
      if (((el | (ba >> 3)) & mid) == mid) x10 = xsign2(x10, 0x80000000u);
      if (((el | (bb >> 3)) & mid) == mid) x01 = xsign2(x01, 0x80000000u);
      if (((el | ((ba | bb) >> 3)) & mid) == mid) x11 = xsign2(x11, 0x80000000u);
    }
    win_apply<kKB>(B, el, x00, x01);
    win_apply<kKB>(B, el | (ba >> 3), x10, x11);
    if (kAcc) acc_b += nrm4(x00, x10, x01, x11);
    at(lds, e) = x00;
    at(lds, e | ba) = x10;
    at(lds, e | bb) = x01;
    at(lds, e | ba | bb) = x11;
  }
}

template <bool kAcc, int kKA, bool kMid, int kTB, int kT>
__device__ __forceinline__ void window_pair_b(char *lds, uint32_t tid, const WinP &A, const WinP &B, uint32_t mid,
                                              double &acc_a, double &acc_b) {
  switch (B.kind) {
    case kWinPlus: window_pair<kAcc, kKA, kWinPlus, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    case kWinMinus: window_pair<kAcc, kKA, kWinMinus, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    case kWinMasked: window_pair<kAcc, kKA, kWinMasked, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    default: window_pair<kAcc, kKA, kWinMaskedSw, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
  }
}

template <bool kAcc, bool kMid, int kTB, int kT>
__device__ __forceinline__ void window_pair_a(char *lds, uint32_t tid, const WinP &A, const WinP &B, uint32_t mid,
                                              double &acc_a, double &acc_b) {
  switch (A.kind) {
    case kWinPlus: window_pair_b<kAcc, kWinPlus, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    case kWinMinus: window_pair_b<kAcc, kWinMinus, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    case kWinMasked: window_pair_b<kAcc, kWinMasked, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
    default: window_pair_b<kAcc, kWinMaskedSw, kMid, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b); break;
  }
}

// Two windows on different bits, with an optional E / Z between them (its
// local bits `mid`, applied when has_mid: the tile's outer bits satisfy it).
template <bool kAcc, int kTB, int kT>
__device__ __forceinline__ void window_pair_any(char *lds, uint32_t tid, const WinP &A, const WinP &B, bool has_mid,
                                                uint32_t mid, double &acc_a, double &acc_b) {
  if (has_mid) window_pair_a<kAcc, true, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b);
  else window_pair_a<kAcc, false, kTB, kT>(lds, tid, A, B, mid, acc_a, acc_b);
}

// Three consecutive unmasked windows A, B, C on three different local bits:
// octets of elements (all values of the three bits) in registers, each
// window applied to its four pairs in turn; one LDS round for three commands.
template <bool kAcc, int kKA, int kKB, int kKC, int kTB, int kT>
__device__ __forceinline__ void window_triple(char *lds, uint32_t tid, const WinP &A, const WinP &B, const WinP &C,
                                              double *acc) {
  constexpr int kOcts = (1 << kTB) / kT / 8;
  int b0 = A.lb, b1 = B.lb, b2 = C.lb;  // sorted copy for the zero insertions
  if (b0 > b1) { const int t = b0; b0 = b1; b1 = t; }
  if (b1 > b2) { const int t = b1; b1 = b2; b2 = t; }
  if (b0 > b1) { const int t = b0; b0 = b1; b1 = t; }
  const uint32_t ba = 8u << A.lb, bb = 8u << B.lb, bc = 8u << C.lb;
#pragma unroll
  for (int r = 0; r < kOcts; ++r) {
    const uint32_t el = ins0u(ins0u(ins0u(tid + uint32_t(r) * kT, b0), b1), b2), e = el << 3;
    float2 x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = at(lds, e | ((q & 1) ? ba : 0u) | ((q & 2) ? bb : 0u) | ((q & 4) ? bc : 0u));
    // unmasked windows: the element index does not enter
    win_apply<kKA>(A, 0u, x[0], x[1]);
    win_apply<kKA>(A, 0u, x[2], x[3]);
    win_apply<kKA>(A, 0u, x[4], x[5]);
    win_apply<kKA>(A, 0u, x[6], x[7]);
    if (kAcc) acc[0] += nrm4(x[0], x[1], x[2], x[3]) + nrm4(x[4], x[5], x[6], x[7]);
    win_apply<kKB>(B, 0u, x[0], x[2]);
    win_apply<kKB>(B, 0u, x[1], x[3]);
    win_apply<kKB>(B, 0u, x[4], x[6]);
    win_apply<kKB>(B, 0u, x[5], x[7]);
    if (kAcc) acc[1] += nrm4(x[0], x[1], x[2], x[3]) + nrm4(x[4], x[5], x[6], x[7]);
    win_apply<kKC>(C, 0u, x[0], x[4]);
    win_apply<kKC>(C, 0u, x[1], x[5]);
    win_apply<kKC>(C, 0u, x[2], x[6]);
    win_apply<kKC>(C, 0u, x[3], x[7]);
    if (kAcc) acc[2] += nrm4(x[0], x[1], x[2], x[3]) + nrm4(x[4], x[5], x[6], x[7]);
#pragma unroll
    for (int q = 0; q < 8; ++q) at(lds, e | ((q & 1) ? ba : 0u) | ((q & 2) ? bb : 0u) | ((q & 4) ? bc : 0u)) = x[q];
  }
}

template <bool kAcc, int kTB, int kT>
__device__ __forceinline__ void window_triple_any(char *lds, uint32_t tid, const WinP &A, const WinP &B,
                                                  const WinP &C, double *acc) {
  // unmasked windows: kind kWinPlus (0) or kWinMinus (1)
  const int sel = A.kind | (B.kind << 1) | (C.kind << 2);
  constexpr int P = kWinPlus, M = kWinMinus;
  switch (sel) {
    case 0: window_triple<kAcc, P, P, P, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 1: window_triple<kAcc, M, P, P, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 2: window_triple<kAcc, P, M, P, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 3: window_triple<kAcc, M, M, P, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 4: window_triple<kAcc, P, P, M, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 5: window_triple<kAcc, M, P, M, kTB, kT>(lds, tid, A, B, C, acc); break;
    case 6: window_triple<kAcc, P, M, M, kTB, kT>(lds, tid, A, B, C, acc); break;
    default: window_triple<kAcc, M, M, M, kTB, kT>(lds, tid, A, B, C, acc); break;
  }
}

// ---- rounds: runs of commands on a register cube.
// A round header (DK_R) names kC local bits (the cube) and the commands
// after it that run on it: windows without local masks whose mixing bit is
// a cube bit, E and Z on any bits.  Each thread loads the 2^kC amplitudes that share its other
// bits (element el | qb[q], q the cube index), applies the round's commands
// in registers in order, and stores them back: one LDS round trip and one
// barrier for the whole run.
//
// The sign r of t in o1 is not applied: the stored value of o1 is r o1
// (pend, bit j: the amplitudes with cube bit j set carry a factor -1), so
// every window is fa a + t, r fb a + t.  Such a factor is common to both
// amplitudes of a pair of any window on another cube bit and commutes with
// E and Z; a window on cube bit j takes it into its coefficient (b arrives
// as -b); the round applies what is left before it stores the cube.

// The cube positions (bit i: cube bit b[i]) of the local bits in m.
template <int kC>
__device__ __forceinline__ uint32_t cube_part(uint32_t m, const int *b) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kC; ++i) c |= ((m >> b[i]) & 1u) << i;
  return c;
}

// A window on one pair in place: t = fc b, b <- fbr a + t, a <- fa a + t.
// Written as one asm statement with the amplitudes as read-write operands:
// the compiler then keeps every amplitude of the cube in one register
// through the round's command loop (with plain C++ it moves half the cube
// between registers after each window).  Two FP32 products and six FMAs,
// no packed instructions.
__device__ __forceinline__ void pair_update(float2 &a, float2 &b, float2 fc, float fa, float fbr) {
  float t0, t1;
  asm("v_mul_f32 %[t0], %[cy], %[by]\n\t"
      "v_mul_f32 %[t1], %[cy], %[bx]\n\t"
      "v_fma_f32 %[t0], %[cx], %[bx], -%[t0]\n\t"
      "v_fma_f32 %[t1], %[cx], %[by], %[t1]\n\t"
      "v_fma_f32 %[bx], %[fb], %[ax], %[t0]\n\t"
      "v_fma_f32 %[by], %[fb], %[ay], %[t1]\n\t"
      "v_fma_f32 %[ax], %[fa], %[ax], %[t0]\n\t"
      "v_fma_f32 %[ay], %[fa], %[ay], %[t1]"
      : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t0] "=&v"(t0), [t1] "=&v"(t1)
      : [cx] "v"(fc.x), [cy] "v"(fc.y), [fa] "v"(fa), [fb] "v"(fbr));
}

// A window on cube bit J (no local masks: rounds hold no masked windows),
// its parameters prepared with the pending sign of position J in fc0 and r
// in fb (prep_window's cs and fold_r).
template <int J, int kC, bool kAcc>
__device__ __forceinline__ double round_window(float2 (&x)[1 << kC], const WinP &w, uint32_t &pend) {
  constexpr int kPer = 1 << kC;
  constexpr int kB = 1 << J;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (q & kB) continue;
    pair_update(x[q], x[q + kB], w.fc0, w.fa, w.fb);
    if (kAcc) acc += nrm2d(x[q], x[q + kB]);
  }
  pend = (pend & ~(1u << J)) | ((w.rsign >> 31) << J);
  return acc;
}

// A composed map on one pair in place: o0 = m00 a + m01 b, o1 = m10 a + m11 b
// (complex entries).  m10 a goes to temporaries first, then a is updated in
// place from the old a and b, then b from the old b: four FP32 products and
// twelve FMAs, with no register moves (one asm statement, as pair_update).
__device__ __forceinline__ void pair_map(float2 &a, float2 &b, float2 m00, float2 m01, float2 m10, float2 m11) {
  float t0, t1, t2, t3;
  asm("v_mul_f32 %[t2], %[m10y], %[ay]\n\t"
      "v_mul_f32 %[t3], %[m10y], %[ax]\n\t"
      "v_fma_f32 %[t2], %[m10x], %[ax], -%[t2]\n\t"
      "v_fma_f32 %[t3], %[m10x], %[ay], %[t3]\n\t"
      "v_mul_f32 %[t0], %[m00y], %[ay]\n\t"
      "v_mul_f32 %[t1], %[m00y], %[ax]\n\t"
      "v_fma_f32 %[ax], %[m00x], %[ax], -%[t0]\n\t"
      "v_fma_f32 %[ay], %[m00x], %[ay], %[t1]\n\t"
      "v_fma_f32 %[ax], %[m01x], %[bx], %[ax]\n\t"
      "v_fma_f32 %[ay], %[m01x], %[by], %[ay]\n\t"
      "v_fma_f32 %[ax], -%[m01y], %[by], %[ax]\n\t"
      "v_fma_f32 %[ay], %[m01y], %[bx], %[ay]\n\t"
      "v_fma_f32 %[t2], -%[m11y], %[by], %[t2]\n\t"
      "v_fma_f32 %[t3], %[m11y], %[bx], %[t3]\n\t"
      "v_fma_f32 %[bx], %[m11x], %[bx], %[t2]\n\t"
      "v_fma_f32 %[by], %[m11x], %[by], %[t3]"
      : [ax] "+v"(a.x), [ay] "+v"(a.y), [bx] "+v"(b.x), [by] "+v"(b.y), [t0] "=&v"(t0), [t1] "=&v"(t1),
        [t2] "=&v"(t2), [t3] "=&v"(t3)
      : [m00x] "v"(m00.x), [m00y] "v"(m00.y), [m01x] "v"(m01.x), [m01y] "v"(m01.y), [m10x] "v"(m10.x),
        [m10y] "v"(m10.y), [m11x] "v"(m11.x), [m11y] "v"(m11.y));
}

// A composed map (DK_U) on cube bit J.  A sign pending on position J means
// the stored b is -b: it negates the column that multiplies b.  The map
// writes o1 whole, so nothing is pending on J after it.
template <int J, int kC>
__device__ __forceinline__ void round_map(float2 (&x)[1 << kC], const FuseOp &op, uint32_t &pend) {
  constexpr int kPer = 1 << kC;
  constexpr int kB = 1 << J;
  const uint32_t s = ((pend >> J) & 1u) << 31;
  const float2 m00 = make_float2(in_vgpr(op.coef.x), in_vgpr(op.coef.y));
  const float2 m01 = make_float2(in_vgpr(__uint_as_float(op.lmask_o1 ^ s)), in_vgpr(__uint_as_float(op.rw_rs ^ s)));
  const float2 m10 = make_float2(in_vgpr(__uint_as_float(op.rw_fa)), in_vgpr(__uint_as_float(op.rw_fbr)));
  const float2 m11 = make_float2(in_vgpr(__uint_as_float(op.rw_cs ^ s)), in_vgpr(__uint_as_float(op.rw_fold ^ s)));
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (q & kB) continue;
    pair_map(x[q], x[q + kB], m00, m01, m10, m11);
  }
  pend &= ~(1u << J);
}

// E or Z in a round: negate the amplitudes whose local bits m are all set
// (the bits outside the cube decide per thread, the cube bits per q: a
// uniform branch per q, so only the amplitudes it can flip are touched).
// e8: the thread's byte offset in the tile (its local index times 8).
template <int kC>
__device__ __forceinline__ void round_diag(float2 (&x)[1 << kC], uint32_t e8, uint32_t m, uint32_t cmask,
                                           const int *b) {
  const uint32_t mr8 = (m & ~cmask) << 3, cm = cube_part<kC>(m, b);
  const uint32_t neg = (e8 & mr8) == mr8 ? 0x80000000u : 0u;
#pragma unroll
  for (int q = 0; q < (1 << kC); ++q)
    if ((uint32_t(q) & cm) == cm) x[q] = xsign2(x[q], neg);  // uniform condition
}

// The round whose header holds `bits` (entries ops[o0 .. o0 + n)): a
// sequence of sweeps, each a header (DK_S: the count of its E / Z and the
// positions of its windows), its E / Z, then its windows in position order.
// Each position has its own code path, so the amplitudes stay in their
// registers through the round.
template <int kTB, bool kRed, bool kMaps>
__device__ __forceinline__ void tile_round(char *lds, uint32_t tid, const FuseOp *__restrict__ ops, int o0, int n,
                                           uint32_t bits, uint64_t ob, const TileArgs &ta,
                                           double (*wacc)[tile_threads(kTB) / 64]) {
  constexpr int kC = tile_cube_bits(kTB);
  constexpr int kPer = 1 << kC;
  static_assert(kPer * tile_threads(kTB) == (1 << kTB), "a thread holds one cube per round");
  const int lane = tid & 63, wave = tid >> 6;
  int b[kC];
  uint32_t cmask = 0;
#pragma unroll
  for (int i = 0; i < kC; ++i) {
    b[i] = int((bits >> (8 * i)) & 0xFFu);
    cmask |= 1u << b[i];
  }
  uint32_t el = tid;
#pragma unroll
  for (int i = 0; i < kC; ++i) el = ins0u(el, b[i]);  // ascending bits
  uint32_t qb[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kC; ++i) v |= uint32_t((q >> i) & 1) << b[i];
    qb[q] = v;
  }
  // the thread's byte offset, hidden from the compiler so that each
  // amplitude's address stays one OR with a uniform word (it would fold the
  // shift back into every address otherwise)
  uint32_t e8 = el << 3;
  opaque32(e8);
  float2 x[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) x[q] = at(lds, e8 | (qb[q] << 3));
  uint32_t pend = 0;
  // one window of the sweep on position J: its norm into wacc (kRed)
  auto window = [&](auto jc, const FuseOp &op) {
    constexpr int J = decltype(jc)::value;
    if constexpr (kMaps) {  // every window slot holds a composed map (passes without window sums)
      round_map<J, kC>(x, op, pend);
    } else {
      const WinP w = prep_window(op, ob, ta, ((pend >> J) & 1u) << 31, true);
      if (kRed) {
        const double d = wave_sum_to_last(round_window<J, kC, true>(x, w, pend));
        if (lane == 63) wacc[w.widx][wave] += d;
      } else {
        round_window<J, kC, false>(x, w, pend);
      }
    }
  };
  for (int o = o0; o < o0 + n;) {
    const FuseOp h = load_op(ops, o++);
    const uint32_t pm = h.flags;
    for (int d = 0; d < h.m_index; ++d) {
      const FuseOp e = load_op(ops, o++);
      if ((ob & e.omask_b) == e.omask_b) round_diag<kC>(x, e8, e.lmask_b, cmask, b);
    }
    if (pm & 1u) window(std::integral_constant<int, 0>(), load_op(ops, o++));
    if (pm & 2u) window(std::integral_constant<int, 1>(), load_op(ops, o++));
    if (pm & 4u) window(std::integral_constant<int, 2>(), load_op(ops, o++));
    if (kC > 3 && (pm & 8u)) window(std::integral_constant<int, (kC > 3 ? 3 : 0)>(), load_op(ops, o++));
  }
#pragma unroll
  for (int j = 0; j < kC; ++j) {
    if ((pend >> j) & 1u) {
#pragma unroll
      for (int q = 0; q < kPer; ++q)
        if (q & (1 << j)) x[q] = xsign2(x[q], 0x80000000u);
    }
  }
  opaque32(e8);  // the store recomputes its addresses: they are not held over the commands
#pragma unroll
  for (int q = 0; q < kPer; ++q) at(lds, e8 | (qb[q] << 3)) = x[q];
}

// The global bit of each tile bit above the thread index (tile bits
// log2(threads) .. kTB-1, lowest first).
template <int kTB>
__device__ __forceinline__ void tile_high_bits(uint64_t tmask, uint64_t *hp) {
  constexpr int kLogT = log2_threads(tile_threads(kTB));
  uint64_t m = tmask;
  for (int i = 0; i < kLogT; ++i) m &= m - 1;
#pragma unroll
  for (int j = 0; j < kTB - kLogT; ++j) {
    hp[j] = m & (~m + 1);
    m &= m - 1;
  }
}

// One tile of a group (tile t of the 2^(n-k)): load it into LDS, apply the
// group's commands, store it back.  With `reduce`, every window adds its
// norm per wave into wacc (FP64 from each thread's sum of squares on).
// Returns, with ta.renorm, this thread's part of the squared norm of the
// stored tile (else 0).  g_tid and hp hold the thread's part of the global
// index and the global bits of the tile bits above the thread index (see
// k_tile).  Ends with a barrier: the tile's LDS is free after it.
template <int kTB, bool kRuns, bool kRed, bool kMaps = false>
__device__ __forceinline__ double tile_one(float2 *__restrict__ psi, const TileArgs &ta,
                                           const FuseOp *__restrict__ ops, double sg, uint64_t t, uint64_t g_tid,
                                           const uint64_t *hp, float2 *tile, double (*wacc)[tile_threads(kTB) / 64]) {
  constexpr bool reduce = kRed;  // a compile-time variant: the FP64 sums cost registers
  constexpr int kT = tile_threads(kTB);
  constexpr int kLogT = log2_threads(kT);
  constexpr int kPer = (1 << kTB) / kT;
  constexpr int kHi = kTB - kLogT;  // tile bits above the thread index
  char *const lds = reinterpret_cast<char *>(tile);
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const uint64_t ob = pdep64(t, ta.omask);
  uint64_t gb = ob | g_tid;
  // live width 28 or less: the tile moves through buffer loads and stores
  // (see vec_rsrc)
  const bool narrow = ((ta.tmask | ta.omask) >> 28) == 0;
  const __amdgpu_buffer_rsrc_t rsrc = vec_rsrc(psi);
  {
    float2 v[kPer];
    if (narrow) {
      const uint32_t toff = uint32_t(g_tid) << 3;
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t u = ob;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) u |= hp[j];
        v[r] = buf_ld(rsrc, toff, uint32_t(u) << 3);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t g = gb;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) g |= hp[j];
        v[r] = psi[g];
      }
    }
    if (ta.nwin > 0 && sg != 1.0) {  // sigma, for the group's first window: applied to the whole tile
      const float gs = float(sg);
#pragma unroll
      for (int r = 0; r < kPer; ++r) v[r] = make_float2(gs * v[r].x, gs * v[r].y);
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) tile[tid + r * kT] = v[r];
  }
  __syncthreads();
  for (int o = 0; o < ta.nops; ++o) {
    const FuseOp op = load_op(ops, o);
    if (op.kind == DK_R) {  // a round: its commands in registers
      tile_round<kTB, kRed, kMaps>(lds, tid, ops, o + 1, op.m_index, op.lmask_b, ob, ta, wacc);
      __syncthreads();
      o += op.m_index;
      continue;
    }
    if (kRuns && op.kind == DK_J && (op.lmask_b | op.lmask_o1) == 0 && o + 2 < ta.nops) {
      const FuseOp n1 = load_op(ops, o + 1), n2 = load_op(ops, o + 2);
      if (n1.kind == DK_J && n2.kind == DK_J && (n1.lmask_b | n1.lmask_o1 | n2.lmask_b | n2.lmask_o1) == 0 &&
          n1.lb != op.lb && n2.lb != op.lb && n2.lb != n1.lb) {
        const WinP A = prep_window(op, ob, ta), B = prep_window(n1, ob, ta), C = prep_window(n2, ob, ta);
        double acc[3] = {0.0, 0.0, 0.0};
        if (reduce) {
          window_triple_any<true, kTB, kT>(lds, tid, A, B, C, acc);
          const double da = wave_sum_to_last(acc[0]), db = wave_sum_to_last(acc[1]), dc = wave_sum_to_last(acc[2]);
          if (lane == 63) {
            wacc[A.widx][wave] += da;
            wacc[B.widx][wave] += db;
            wacc[C.widx][wave] += dc;
          }
        } else {
          window_triple_any<false, kTB, kT>(lds, tid, A, B, C, acc);
        }
        __syncthreads();
        o += 2;
        continue;
      }
    }
    if (kRuns && op.kind == DK_J && o + 1 < ta.nops) {
      FuseOp nx = load_op(ops, o + 1);
      // an E or Z between two windows joins them (applied in registers)
      int skip = 1;
      bool has_mid = false;
      uint32_t mid = 0;
      if ((nx.kind == DK_E || nx.kind == DK_Z) && o + 2 < ta.nops) {
        const FuseOp n2 = load_op(ops, o + 2);
        if (n2.kind == DK_J && n2.lb != op.lb) {
          has_mid = (ob & nx.omask_b) == nx.omask_b;
          mid = nx.lmask_b;
          nx = n2;
          skip = 2;
        }
      }
      if (nx.kind == DK_J && nx.lb != op.lb) {
        const WinP A = prep_window(op, ob, ta), B = prep_window(nx, ob, ta);
        double acc_a = 0.0, acc_b = 0.0;
        if (reduce) {
          window_pair_any<true, kTB, kT>(lds, tid, A, B, has_mid, mid, acc_a, acc_b);
          const double da = wave_sum_to_last(acc_a), db = wave_sum_to_last(acc_b);
          if (lane == 63) {
            wacc[A.widx][wave] += da;
            wacc[B.widx][wave] += db;
          }
        } else {
          window_pair_any<false, kTB, kT>(lds, tid, A, B, has_mid, mid, acc_a, acc_b);
        }
        __syncthreads();
        o += skip;
        continue;
      }
    }
    if (op.kind == DK_E || op.kind == DK_Z) {
      if ((ob & op.omask_b) == op.omask_b) diag_flip<kTB, kT>(lds, tid, op.lmask_b);
    } else if (op.kind == DK_X) {
      pair_swap<kTB, kT>(lds, tid, op.lb);
    } else {  // window: fold the tile-constant signs and the corrections
      const WinP w = prep_window(op, ob, ta);
      if (reduce) {
        const double d = wave_sum_to_last(window_single<true, kTB, kT>(lds, tid, w));  // FP64 from the wave sum on
        if (lane == 63) wacc[w.widx][wave] += d;
      } else {
        window_single<false, kTB, kT>(lds, tid, w);
      }
    }
    __syncthreads();
  }
  double rsum = 0.0;
  {
    float2 v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) v[r] = tile[tid + r * kT];
    if (ta.renorm) {  // uniform: the group's output norm resets sigma
#pragma unroll
      for (int r = 0; r < kPer; r += 2) rsum += nrm2d(v[r], v[r + 1]);
    }
    opaque(gb);  // the load's addresses are not kept live over the commands: recomputed here
    if (narrow) {
      const uint32_t toff = uint32_t(g_tid) << 3;
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t u = ob;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) u |= hp[j];
        buf_st(rsrc, toff, uint32_t(u) << 3, v[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t g = gb;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) g |= hp[j];
        psi[g] = v[r];
      }
    }
  }
  __syncthreads();
  return rsum;
}

// Sum of x over the workgroup, valid in thread 0, through `scratch` (one
// double per wave of LDS that no thread uses meanwhile).
template <int kT>
__device__ __forceinline__ double block_sum0(double x, double *scratch) {
  const uint32_t tid = threadIdx.x;
  const double d = wave_sum_to_last(x);
  if ((tid & 63) == 63) scratch[tid >> 6] = d;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int k = 0; k < kT / 64; ++k) s += scratch[k];
  return s;
}

// kTB = tile bits (ta.k).  Global memory <-> LDS: each thread moves
// kPer = 2^kTB / kT amplitudes per tile, all loads issued before the first
// LDS store (and all LDS reads before the first global store), so the memory
// system sees kPer requests in flight per thread.  Element e of the tile
// whose outer bits are `ob` sits at global index ob | pdep(e, tmask); with
// e = tid + r kT that is ob | pdep(tid, tmask) | (a uniform part from r).
// Every command of the group is then one pass over the tile in LDS.
// kRuns: the run-in-registers paths are compiled in (they raise the VGPR
// count, which lowers occupancy for groups that cannot use them).
template <int kTB, bool kRuns, bool kRed, bool kMaps = false>
__global__ __launch_bounds__(tile_threads(kTB)) void k_tile(float2 *__restrict__ psi, TileArgs ta,
                                                            const FuseOp *__restrict__ ops, MeasureArgs ma,
                                                            double *__restrict__ partials) {
  constexpr int kT = tile_threads(kTB);
  constexpr int kHi = kTB - log2_threads(kT);  // tile bits above the thread index
  __shared__ float2 tile[1 << kTB];
  __shared__ double wacc[kMaxGroupWindows][kT / 64];
  const uint32_t tid = threadIdx.x;
  constexpr bool reduce = kRed;  // ma.reduce != kReduceNone
  if (reduce)
    for (int i = tid; i < ta.nwin * (kT / 64); i += kT) wacc[i / (kT / 64)][i % (kT / 64)] = 0.0;
  const double sg = (ma.reduce == kReduceRenorm) ? *ma.book.sigma : 1.0;
  const uint64_t g_tid = pdep64(tid, ta.tmask);
  uint64_t hp[kHi];
  tile_high_bits<kTB>(ta.tmask, hp);
  psi += size_t(blockIdx.y) * ta.set_stride;
  if (ta.half_m && blockIdx.x == 0 && blockIdx.y == 0)  // windows with p = 1/2 exactly
    for (int i = tid; i < ta.nwin; i += kT) ma.book.probs[ta.half_m[i]] = 0.5;
  const uint64_t ntiles = uint64_t(1) << (ta.n - kTB);
  double rsum = 0.0;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
    rsum += tile_one<kTB, kRuns, kRed, kMaps>(psi, ta, ops, sg, t, g_tid, hp, tile, wacc);
  if (ta.renorm) {  // the block's share of the output norm, summed through the free tile LDS
    const double sum = block_sum0<kT>(rsum, reinterpret_cast<double *>(tile));
    if (tid == 0) partials[blockIdx.x] = sum;
  }
  if (reduce) {
    for (int w = tid; w < ta.nwin; w += kT) {
      double s = 0.0;
      for (int k = 0; k < kT / 64; ++k) s += wacc[w][k];
      partials[size_t(w) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// A row of a read-only device table, loaded whole through scalar loads (the
// index is uniform over the workgroup; the table is never written by a
// kernel, so the constant address space may be used).
template <typename T>
__device__ __forceinline__ T load_row(const T *tab, uint32_t i) {
  static_assert(sizeof(T) % 4 == 0, "table rows are whole dwords");
  constexpr int kW = sizeof(T) / 4;
  typedef const __attribute__((address_space(4))) uint32_t cword;
  cword *src = reinterpret_cast<cword *>(reinterpret_cast<uintptr_t>(tab)) +
               size_t(kW) * __builtin_amdgcn_readfirstlane(i);
  uint32_t w[kW];
#pragma unroll
  for (int k = 0; k < kW; ++k) w[k] = src[k];
  T v;
  __builtin_memcpy(&v, w, sizeof(v));
  return v;
}

__device__ __forceinline__ uint32_t first_tile_of(const MultiTile *ents, int e) {
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const uintptr_t a = reinterpret_cast<uintptr_t>(ents + __builtin_amdgcn_readfirstlane(e)) +
                      offsetof(MultiTile, first_tile);
  return *reinterpret_cast<cword *>(a);
}

// Tile groups of many patterns in one launch (batched runs): the grid walks
// the concatenated tiles of all entries; a workgroup finds the entry that
// owns its tile (binary search on first_tile), runs that tile as k_tile
// does, and stores its windows' sums per tile (partials[w * ntiles + t]), so
// that k_finish_multi sums them in tile order.
template <int kTB, bool kRuns, bool kRed, bool kMaps = false>
__global__ __launch_bounds__(tile_threads(kTB)) void k_tile_multi(const MultiTile *__restrict__ ents, int nent,
                                                                  uint32_t total) {
  constexpr int kT = tile_threads(kTB);
  constexpr int kHi = kTB - log2_threads(kT);
  __shared__ float2 tile[1 << kTB];
  __shared__ double wacc[kMaxGroupWindows][kT / 64];
  const uint32_t tid = threadIdx.x;
  for (uint32_t gt = blockIdx.x; gt < total; gt += gridDim.x) {
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first_tile_of(ents, mid) <= gt) lo = mid;
      else hi = mid - 1;
    }
    const MultiTile e = load_row(ents, uint32_t(lo));
    const uint64_t t = gt - e.first_tile;
    constexpr bool reduce = kRed;  // every entry of the launch: e.reduce != kReduceNone
    if (reduce)
      for (int i = tid; i < e.ta.nwin * (kT / 64); i += kT) wacc[i / (kT / 64)][i % (kT / 64)] = 0.0;
    const double sg = e.reduce == kReduceRenorm ? *e.sigma : 1.0;
    const uint64_t g_tid = pdep64(tid, e.ta.tmask);
    uint64_t hp[kHi];
    tile_high_bits<kTB>(e.ta.tmask, hp);
    if (e.ta.half_m && t == 0)  // windows with p = 1/2 exactly
      for (int i = tid; i < e.ta.nwin; i += kT) e.probs[e.ta.half_m[i]] = 0.5;
    const double rsum = tile_one<kTB, kRuns, kRed, kMaps>(e.psi, e.ta, e.ops, sg, t, g_tid, hp, tile, wacc);
    if (e.ta.renorm) {  // the tile's output norm, summed through the free tile LDS
      const double sum = block_sum0<kT>(rsum, reinterpret_cast<double *>(tile));
      if (tid == 0) e.partials[t] = sum;
      __syncthreads();  // the next tile's loads overwrite the LDS
    }
    if (reduce) {
      const uint64_t ntiles = uint64_t(1) << (e.ta.n - kTB);
      for (int w = tid; w < e.ta.nwin; w += kT) {
        double sum = 0.0;
        for (int k = 0; k < kT / 64; ++k) sum += wacc[w][k];
        e.partials[size_t(w) * ntiles + t] = sum;
      }
      __syncthreads();  // wacc is cleared for the next tile
    }
  }
}

// Reverse sweep of a window on the element pairs that differ in local bit
// lb, for the psi tile (output -> input) and the lambda tile (after -> before)
// at once; windows must have an odd number of E between their qubits.  In
// the window's own terms (see k_b_window_rev): o0 = f (a + sb c b),
// o1 = so1 f (a - sb c b), then the folded corrections P; the pair's signs
// sb, so1 are the parities of its local bits under lmb / lmo times the
// tile-constant parities osb / oso of the outer bits.  Returns this thread's
// sum of 2 Re <lambda | dW/dtheta psi_in>.
template <int kTB, int kT>
__device__ __forceinline__ double window_rev(char *lp, char *ll, uint32_t tid, int lb, float f, float2 c, uint32_t lmb,
                                             uint32_t lmo, float osb, float oso, bool swap, bool neg0, bool neg1) {
  constexpr int kPairs = (1 << kTB) / kT / 2;
  const uint32_t et = ins0u(tid, lb), bit8 = 8u << lb;
  const float2 cc = make_float2(c.x, -c.y);
  const float g = 0.5f / f;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kPairs; ++r) {
    const uint32_t ur = ins0u(uint32_t(r) * kT, lb);
    const uint32_t e0 = et | ur, a0 = e0 << 3, a1 = a0 | bit8;
    const float sb = par32(e0 & lmb) ? -osb : osb, so1 = par32(e0 & lmo) ? -oso : oso;
    float2 o0 = *reinterpret_cast<const float2 *>(lp + a0), o1 = *reinterpret_cast<const float2 *>(lp + a1);
    if (neg0) o0 = make_float2(-o0.x, -o0.y);
    if (neg1) o1 = make_float2(-o1.x, -o1.y);
    if (swap) { const float2 t = o0; o0 = o1; o1 = t; }
    const float2 pa = make_float2(g * (o0.x + so1 * o1.x), g * (o0.y + so1 * o1.y));
    const float2 dd = make_float2(o0.x - so1 * o1.x, o0.y - so1 * o1.y);
    const float2 pd = make_float2(cc.x * dd.x - cc.y * dd.y, cc.x * dd.y + cc.y * dd.x);
    const float2 pb = make_float2(g * sb * pd.x, g * sb * pd.y);
    const float2 cb = make_float2(c.x * pb.x - c.y * pb.y, c.x * pb.y + c.y * pb.x);
    const float g0 = f * sb, g1 = -so1 * f * sb;
    float2 d0 = make_float2(g0 * cb.y, -g0 * cb.x), d1 = make_float2(g1 * cb.y, -g1 * cb.x);
    if (swap) { const float2 t = d0; d0 = d1; d1 = t; }
    if (neg0) d0 = make_float2(-d0.x, -d0.y);
    if (neg1) d1 = make_float2(-d1.x, -d1.y);
    const float2 l0 = *reinterpret_cast<const float2 *>(ll + a0), l1 = *reinterpret_cast<const float2 *>(ll + a1);
    acc += 2.0 * (double(l0.x) * d0.x + double(l0.y) * d0.y + double(l1.x) * d1.x + double(l1.y) * d1.y);
    float2 m0 = neg0 ? make_float2(-l0.x, -l0.y) : l0;
    float2 m1 = neg1 ? make_float2(-l1.x, -l1.y) : l1;
    if (swap) { const float2 t = m0; m0 = m1; m1 = t; }
    const float2 sm = make_float2(m0.x + so1 * m1.x, m0.y + so1 * m1.y);
    const float2 dm = make_float2(m0.x - so1 * m1.x, m0.y - so1 * m1.y);
    const float2 cd = make_float2(cc.x * dm.x - cc.y * dm.y, cc.x * dm.y + cc.y * dm.x);
    *reinterpret_cast<float2 *>(lp + a0) = pa;
    *reinterpret_cast<float2 *>(lp + a1) = pb;
    *reinterpret_cast<float2 *>(ll + a0) = make_float2(f * sm.x, f * sm.y);
    *reinterpret_cast<float2 *>(ll + a1) = make_float2(f * sb * cd.x, f * sb * cd.y);
  }
  return acc;
}

// The reverse of a tile group on set blockIdx.y: the psi and lambda tiles sit
// side by side in LDS and the commands run last to first (E, X, Z are their
// own inverses and adjoints).
template <int kTB>
__global__ __launch_bounds__(tile_threads(kTB)) void k_tile_rev(float2 *__restrict__ psi, float2 *__restrict__ lam,
                                                                TileArgs ta, const FuseOp *__restrict__ ops,
                                                                double *__restrict__ partials, int q_first,
                                                                unsigned nblk) {
  constexpr int kT = tile_threads(kTB);
  constexpr int kLogT = log2_threads(kT);
  constexpr int kPer = (1 << kTB) / kT;
  constexpr int kHi = kTB - kLogT;
  extern __shared__ float2 tile[];
  __shared__ double wacc[kMaxGroupWindows][kT / 64];
  char *const lp = reinterpret_cast<char *>(tile);
  char *const ll = reinterpret_cast<char *>(tile + (1 << kTB));
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < ta.nwin * (kT / 64); i += kT) wacc[i / (kT / 64)][i % (kT / 64)] = 0.0;
  psi += size_t(blockIdx.y) * ta.set_stride;
  lam += size_t(blockIdx.y) * ta.set_stride;
  const uint64_t g_tid = pdep64(tid, ta.tmask);
  uint64_t hp[kHi];
  {
    uint64_t m = ta.tmask;
    for (int i = 0; i < kLogT; ++i) m &= m - 1;
#pragma unroll
    for (int j = 0; j < kHi; ++j) {
      hp[j] = m & (~m + 1);
      m &= m - 1;
    }
  }
  const uint64_t ntiles = uint64_t(1) << (ta.n - kTB);
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t ob = pdep64(t, ta.omask);
    const uint64_t gb = ob | g_tid;
    {
      float2 v[kPer], w[kPer];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t g = gb;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) g |= hp[j];
        v[r] = psi[g];
        w[r] = lam[g];
      }
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        tile[tid + r * kT] = v[r];
        tile[(1 << kTB) + tid + r * kT] = w[r];
      }
    }
    __syncthreads();
    for (int o = ta.nops - 1; o >= 0; --o) {
      const FuseOp op = load_op(ops, o);
      if (op.kind == DK_R || op.kind == DK_S) continue;  // round and sweep headers: one command at a time here
      if (op.kind == DK_E || op.kind == DK_Z) {
        if ((ob & op.omask_b) == op.omask_b) {
          diag_flip<kTB, kT>(lp, tid, op.lmask_b);
          diag_flip<kTB, kT>(ll, tid, op.lmask_b);
        }
      } else if (op.kind == DK_X) {
        pair_swap<kTB, kT>(lp, tid, op.lb);
        pair_swap<kTB, kT>(ll, tid, op.lb);
      } else {
        const float2 cw = set_coef(ta, op.m_index);
        const float osb = par64(ob & op.omask_b) ? -1.f : 1.f, oso = par64(ob & op.omask_o1) ? -1.f : 1.f;
        const double acc = window_rev<kTB, kT>(lp, ll, tid, op.lb, op.f, cw, op.lmask_b, op.lmask_o1, osb, oso,
                                               op.flags & 1u, op.flags & 2u, op.flags & 4u);
        const double d = wave_sum_to_last(acc);
        if (lane == 63) wacc[op.widx][wave] += d;
      }
      __syncthreads();
    }
    {
      float2 v[kPer], w[kPer];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        v[r] = tile[tid + r * kT];
        w[r] = tile[(1 << kTB) + tid + r * kT];
      }
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        uint64_t g = gb;
#pragma unroll
        for (int j = 0; j < kHi; ++j)
          if ((r >> j) & 1) g |= hp[j];
        psi[g] = v[r];
        lam[g] = w[r];
      }
    }
    __syncthreads();
  }
  for (int w = tid; w < ta.nwin; w += kT) {
    double s = 0.0;
    for (int k = 0; k < kT / 64; ++k) s += wacc[w][k];
    partials[((size_t(q_first) + w) * ta.nsets + blockIdx.y) * nblk + blockIdx.x] = s;
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

// After a group whose windows all have p = 1/2 and which ends a run of
// them (TileArgs::renorm): sigma = 1 / sqrt(n), n the squared norm of the
// group's output summed from the per-block partials in block order.
__global__ __launch_bounds__(kTT) void k_finish_renorm(DevBook book, unsigned nblk) {
  const double n = sum_partials(book.partials, nblk);
  if (threadIdx.x == 0) *book.sigma = n > 1e-300 ? 1.0 / sqrt(n) : 0.0;
}

// The group finish of many patterns at once: block (g, e) does for window
// g of entry e what k_finish_group does, with the entry's per-tile partials
// (an entry with renorm: block (0, e) does what k_finish_renorm does).
__global__ __launch_bounds__(kTT) void k_finish_multi(const MultiFinish *__restrict__ fins) {
  const MultiFinish f = load_row(fins, blockIdx.y);
  const int g = blockIdx.x;
  if (g >= f.nwin) return;  // uniform over the block
  if (f.renorm) {
    const double n = sum_partials(f.book.partials, f.ntiles);
    if (threadIdx.x == 0) *f.book.sigma = n > 1e-300 ? 1.0 / sqrt(n) : 0.0;
    return;
  }
  const double n = sum_partials(f.book.partials + size_t(g) * f.ntiles, f.ntiles);
  const double prev = g > 0 ? sum_partials(f.book.partials + size_t(g - 1) * f.ntiles, f.ntiles) : 1.0;
  if (threadIdx.x != 0) return;
  const double p = prev > 0.0 ? 0.5 * n / prev : 0.0;
  const int m = f.m_of_window[g];
  f.book.probs[m] = p;
  if (f.reduce == kReduceRenorm && p < 1e-10) {
    atomicMin(&f.book.err[0], m);
    f.book.err[1] = kErrZeroProb;
  } else if (f.reduce == kReduceCheck && fabs(p - 0.5) > 1e-4) {
    atomicMin(&f.book.err[0], m);
    f.book.err[1] = kErrNotDet;
  }
  if (f.reduce == kReduceRenorm && g == f.nwin - 1) *f.book.sigma = n > 1e-300 ? 1.0 / sqrt(n) : 0.0;
}

}  // namespace

// One workgroup per tile up to kTileGridCap tiles (measured best for 2^12
// tiles of 2^12 amplitudes: 3.2 rounds of workgroups at five a CU); beyond
// that 2048 workgroups loop over the tiles (for 2^13 tiles of 2^11, one
// round of workgroups with four tiles each beats 4096 with two).
unsigned tile_grid(const TileArgs &ta) {
  const uint64_t ntiles = uint64_t(1) << (ta.n - ta.k);
  return unsigned(ntiles <= kTileGridCap ? ntiles : 2048u);
}

namespace {

// Dynamic LDS limits of every tile kernel with 2^kTB-amplitude tiles.
template <int kTB>
hipError_t prepare_bits() {
  const int one = int(sizeof(float2) << kTB), two = 2 * one;
  const void *fns[] = {
      reinterpret_cast<const void *>(k_tile<kTB, false, false>), reinterpret_cast<const void *>(k_tile<kTB, false, true>),
      reinterpret_cast<const void *>(k_tile<kTB, true, false>), reinterpret_cast<const void *>(k_tile<kTB, true, true>),
      reinterpret_cast<const void *>(k_tile<kTB, false, false, true>),
      reinterpret_cast<const void *>(k_tile<kTB, true, false, true>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, false, false>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, false, true>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, true, false>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, true, true>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, false, false, true>),
      reinterpret_cast<const void *>(k_tile_multi<kTB, true, false, true>)};
  hipError_t e = hipSuccess;
  for (const void *f : fns)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, one);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_rev<kTB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, two);
  return e;
}

// One tile pass: the instance compiled for these tile bits, register runs
// (ta.runs) and reduction (FP64 window sums).
template <int kTB>
void tile_launch(bool runs, bool red, dim3 grid, hipStream_t s, float2 *psi, const TileArgs &ta, const FuseOp *ops,
                 const MeasureArgs &a, double *partials) {
  const dim3 block(tile_threads(kTB));
  if (ta.maps && !red) {  // rounds of composed maps only
    if (runs) hipLaunchKernelGGL((k_tile<kTB, true, false, true>), grid, block, 0, s, psi, ta, ops, a, partials);
    else hipLaunchKernelGGL((k_tile<kTB, false, false, true>), grid, block, 0, s, psi, ta, ops, a, partials);
    return;
  }
  if (runs) {
    if (red) hipLaunchKernelGGL((k_tile<kTB, true, true>), grid, block, 0, s, psi, ta, ops, a, partials);
    else hipLaunchKernelGGL((k_tile<kTB, true, false>), grid, block, 0, s, psi, ta, ops, a, partials);
  } else {
    if (red) hipLaunchKernelGGL((k_tile<kTB, false, true>), grid, block, 0, s, psi, ta, ops, a, partials);
    else hipLaunchKernelGGL((k_tile<kTB, false, false>), grid, block, 0, s, psi, ta, ops, a, partials);
  }
}

template <int kTB>
void tile_multi_launch(bool runs, bool red, bool maps, dim3 grid, hipStream_t s, const MultiTile *ents, int nent,
                       uint32_t total) {
  const dim3 block(tile_threads(kTB));
  if (maps && !red) {  // every entry's rounds hold composed maps only
    if (runs) hipLaunchKernelGGL((k_tile_multi<kTB, true, false, true>), grid, block, 0, s, ents, nent, total);
    else hipLaunchKernelGGL((k_tile_multi<kTB, false, false, true>), grid, block, 0, s, ents, nent, total);
    return;
  }
  if (runs) {
    if (red) hipLaunchKernelGGL((k_tile_multi<kTB, true, true>), grid, block, 0, s, ents, nent, total);
    else hipLaunchKernelGGL((k_tile_multi<kTB, true, false>), grid, block, 0, s, ents, nent, total);
  } else {
    if (red) hipLaunchKernelGGL((k_tile_multi<kTB, false, true>), grid, block, 0, s, ents, nent, total);
    else hipLaunchKernelGGL((k_tile_multi<kTB, false, false>), grid, block, 0, s, ents, nent, total);
  }
}

}  // namespace

hipError_t tile_prepare() {
  hipError_t e = prepare_bits<10>();
  if (e == hipSuccess) e = prepare_bits<11>();
  if (e == hipSuccess) e = prepare_bits<12>();
  if (e == hipSuccess) e = prepare_bits<13>();
  return e;
}

hipError_t launch_tile(float2 *psi, const TileArgs &ta, const FuseOp *ops, const MeasureArgs &a, hipStream_t s,
                       unsigned *grid) {
  // the per-window sums hold kMaxGroupWindows; larger groups only run without them
  const bool red = a.reduce != kReduceNone;
  if (ta.nwin > (red ? kMaxGroupWindows : kMaxHalfWindows)) return hipErrorInvalidValue;
  const unsigned g = tile_grid(ta);
  switch (ta.k) {
    case 10: tile_launch<10>(ta.runs, red, dim3(g), s, psi, ta, ops, a, a.book.partials); break;
    case 11: tile_launch<11>(ta.runs, red, dim3(g), s, psi, ta, ops, a, a.book.partials); break;
    case 12: tile_launch<12>(ta.runs, red, dim3(g), s, psi, ta, ops, a, a.book.partials); break;
    case 13: tile_launch<13>(ta.runs, red, dim3(g), s, psi, ta, ops, a, a.book.partials); break;
    default: return hipErrorInvalidValue;
  }
  *grid = g;
  return hipGetLastError();
}

hipError_t launch_tile_sets(float2 *psi, const TileArgs &ta0, const FuseOp *ops, int nsets, size_t set_stride,
                            const float2 *coefs, hipStream_t s) {
  TileArgs ta = ta0;
  ta.set_stride = set_stride;
  ta.coefs = coefs;
  ta.nsets = nsets;
  MeasureArgs a{};
  a.reduce = kReduceNone;
  const dim3 grid(tile_grid(ta), unsigned(nsets));
  switch (ta.k) {
    case 10: tile_launch<10>(ta.runs, false, grid, s, psi, ta, ops, a, nullptr); break;
    case 11: tile_launch<11>(ta.runs, false, grid, s, psi, ta, ops, a, nullptr); break;
    case 12: tile_launch<12>(ta.runs, false, grid, s, psi, ta, ops, a, nullptr); break;
    case 13: tile_launch<13>(ta.runs, false, grid, s, psi, ta, ops, a, nullptr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile_rev(float2 *psi, float2 *lam, const TileArgs &ta0, const FuseOp *ops, int nsets,
                           size_t set_stride, const float2 *coefs, double *partials, int q_first, unsigned nblk,
                           hipStream_t s) {
  if (ta0.nwin > kMaxGroupWindows) return hipErrorInvalidValue;  // its per-window sums hold that many
  TileArgs ta = ta0;
  ta.set_stride = set_stride;
  ta.coefs = coefs;
  ta.nsets = nsets;
  const size_t bytes = 2 * sizeof(float2) << ta.k;
  const dim3 grid(tile_grid(ta), unsigned(nsets));
  if (grid.x > nblk) return hipErrorInvalidValue;  // the partials rows hold nblk blocks
  switch (ta.k) {
    case 10: hipLaunchKernelGGL(k_tile_rev<10>, grid, dim3(tile_threads(10)), bytes, s, psi, lam, ta, ops, partials, q_first, nblk); break;
    case 11: hipLaunchKernelGGL(k_tile_rev<11>, grid, dim3(tile_threads(11)), bytes, s, psi, lam, ta, ops, partials, q_first, nblk); break;
    case 12: hipLaunchKernelGGL(k_tile_rev<12>, grid, dim3(tile_threads(12)), bytes, s, psi, lam, ta, ops, partials, q_first, nblk); break;
    case 13: hipLaunchKernelGGL(k_tile_rev<13>, grid, dim3(tile_threads(13)), bytes, s, psi, lam, ta, ops, partials, q_first, nblk); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile_multi(const MultiTile *ents, int nent, uint32_t total, int k, bool runs, bool red,
                             bool maps, hipStream_t s) {
  if (nent <= 0 || total == 0) return hipGetLastError();
  const dim3 grid(total < 65535u ? total : 65535u);
  switch (k) {
    case 10: tile_multi_launch<10>(runs, red, maps, grid, s, ents, nent, total); break;
    case 11: tile_multi_launch<11>(runs, red, maps, grid, s, ents, nent, total); break;
    case 12: tile_multi_launch<12>(runs, red, maps, grid, s, ents, nent, total); break;
    case 13: tile_multi_launch<13>(runs, red, maps, grid, s, ents, nent, total); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finish_multi(const MultiFinish *fins, int nfin, int maxwin, hipStream_t s) {
  if (nfin <= 0 || maxwin <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_finish_multi, dim3(unsigned(maxwin), unsigned(nfin)), dim3(kTT), 0, s, fins);
  return hipGetLastError();
}

hipError_t launch_finish_renorm(const DevBook &book, unsigned nblk, hipStream_t s) {
  if (nblk == 0 || nblk > kTileGridCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish_renorm, dim3(1), dim3(kTT), 0, s, book, nblk);
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
