// owqs_host.cpp -- the C ABI of libowqs (include/owqs.h): pattern loading and
// validation, the host plan compiler and the run / read entry points.
//
// The plan compiler walks the command list once per (angles, outcomes, mode,
// exec) setting and emits one device step per non-trivial command:
//   - qubit ids map to slots (index bits).  Inputs take slots 0..nin-1; N puts
//     the new qubit on the top slot; M moves the top qubit into the measured
//     slot (the kernels' in-place layout), so the vector stays contiguous;
//   - signals are resolved with the forced outcomes: theta = (-1)^s alpha +
//     t pi (Eq. 2) and the kernel coefficient c = (-1)^o e^{-i theta}
//     (Eqs. 11-12) is computed in FP64 and rounded to complex64; X/Z with a
//     zero signal emit nothing;
//   - the 1/sqrt 2 of every N stays a host factor until the next M folds it
//     into its pass (with the device FP64 sigma in OWQS mode).
#include <array>
#include <atomic>

#include "owqs_host_impl.h"
#include "owqs_pattern_access.h"

namespace owqs {

owqs_status fail(owqs_ctx *ctx, owqs_status st, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

owqs_status hip_fail(owqs_ctx *ctx, hipError_t e, const char *what) {
  return fail(ctx, OWQS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Validate D0-D3 (Sec. 2.2) and compute the largest live width.
owqs_status validate(owqs_pattern *p) {
  enum { UNPREP = 0, LIVE = 1, MEAS = 2 };
  std::vector<int> st(p->nq, UNPREP);
  std::vector<char> is_out(p->nq, 0);
  for (int q : p->outputs) {
    if (is_out[q]) return fail(p->ctx, OWQS_E_INVALID_ARG, "duplicate output qubit");
    is_out[q] = 1;
  }
  for (int q : p->inputs) {
    if (st[q] != UNPREP) return fail(p->ctx, OWQS_E_INVALID_ARG, "duplicate input qubit");
    st[q] = LIVE;
  }
  int n = (int)p->inputs.size(), m = n, meas = 0;
  for (size_t i = 0; i < p->cmds.size(); ++i) {
    const Cmd &c = p->cmds[i];
    auto bad = [&](const char *why) {
      return fail(p->ctx, OWQS_E_PATTERN, "command " + std::to_string(i) + ": " + why);
    };
    switch (c.op) {
      case OWQS_OP_N:
        if (st[c.q0] != UNPREP) return bad("N on a qubit that is an input or already prepared (D2)");
        st[c.q0] = LIVE;
        ++n;
        if (n > m) m = n;
        break;
      case OWQS_OP_E:
        if (c.q0 == c.q1) return bad("E on a single qubit");
        if (st[c.q0] != LIVE || st[c.q1] != LIVE) return bad("E on a qubit not live (D1/D2)");
        break;
      case OWQS_OP_M:
      case OWQS_OP_X:
      case OWQS_OP_Z:
        if (st[c.q0] != LIVE) return bad("action on a qubit not live (D1/D2)");
        for (int j : c.s)
          if (st[j] != MEAS) return bad("signal depends on an unmeasured qubit (D0)");
        for (int j : c.t)
          if (st[j] != MEAS) return bad("signal depends on an unmeasured qubit (D0)");
        if (c.op == OWQS_OP_M) {
          if (is_out[c.q0]) return bad("an output qubit is measured (D3)");
          st[c.q0] = MEAS;
          --n;
          ++meas;
        }
        break;
      default:
        return bad("unknown opcode");
    }
  }
  for (int q = 0; q < p->nq; ++q) {
    if (is_out[q] && st[q] != LIVE) return fail(p->ctx, OWQS_E_PATTERN, "an output qubit is not live at the end (D3)");
    if (!is_out[q] && st[q] == LIVE) return fail(p->ctx, OWQS_E_PATTERN, "a non-output qubit is never measured (D3)");
  }
  p->n_meas = meas;
  p->max_live = m;
  return OWQS_OK;
}

int signal(const std::vector<int> &dom, const std::vector<int> &outcome_of) {
  int s = 0;
  for (int j : dom) s ^= outcome_of[j];
  return s;
}

// Whether two window/E/X/Z steps at one width may swap: neither mixes a slot
// (a window's or an X's) that the other mixes or reads as a sign (E and Z
// slots, a window's masks), and they are not two windows whose probability
// depends on the state (an even E(v, w) count): swapping those would change
// what each records.  Windows with an odd count act as a unitary times 1/2
// of the norm, so the other's probability is the same on either side.
bool commute_steps(const Step &a, const Step &b) {
  auto mix = [](const Step &x) -> uint64_t {
    return (x.kind == S_J || x.kind == S_X) ? uint64_t(1) << x.b0 : 0;
  };
  auto diag = [](const Step &x) -> uint64_t {
    if (x.kind == S_E) return (uint64_t(1) << x.b0) | (uint64_t(1) << x.b1);
    if (x.kind == S_Z) return uint64_t(1) << x.b0;
    if (x.kind == S_J) return x.win.mask_b | x.win.mask_o1;
    return 0;
  };
  if (mix(a) & (mix(b) | diag(b))) return false;
  if (mix(b) & (mix(a) | diag(a))) return false;
  return !(a.kind == S_J && b.kind == S_J && a.win.vw_even && b.win.vw_even);
}

// Order the commands of a tile group (local bits < k) into rounds over
// register cubes of tile_cube_bits(k) bits (see k_tile): a round holds
// windows without local masks on at most that many distinct mixing bits
// and E / Z on any bits,
// in an order that keeps every pair of commands that do not commute (a
// mixing bit of one meets a bit the other mixes or reads) as it was, and,
// unless free_windows, all windows in their order.  Ready commands are taken
// first come first served, each round growing while any ready command fits
// it.  X and masked windows run on their own, and so do E / Z that meet no
// window of a round.
struct RoundItem {
  int op;         // >= 0: a command of the group; -1: a round header; -2: a sweep header
  int count;      // round header: the entries of the round (they follow it); sweep: its E / Z
  uint32_t bits;  // round header: the cube's local bits, one per byte, ascending; sweep: its
                  // window positions (bit p: a window on cube bit p)
};

std::vector<RoundItem> schedule_rounds(const std::vector<FuseOp> &g, int k, bool free_windows) {
  const int kc = tile_cube_bits(k);
  const int n = int(g.size());
  auto mix = [](const FuseOp &o) -> uint32_t { return (o.kind == DK_J || o.kind == DK_X) ? 1u << o.lb : 0u; };
  auto diag = [](const FuseOp &o) -> uint32_t {
    if (o.kind == DK_J) return o.lmask_b | o.lmask_o1;
    if (o.kind == DK_E || o.kind == DK_Z) return o.lmask_b;
    return 0u;
  };
  // windows with local masks run outside rounds (the single and paired
  // window paths), like X
  auto masked = [](const FuseOp &o) { return o.kind == DK_J && (o.lmask_b | o.lmask_o1) != 0; };
  std::vector<std::vector<int>> pred(static_cast<size_t>(n));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      const bool conflict = (mix(g[i]) & (mix(g[j]) | diag(g[j]))) || (mix(g[j]) & (mix(g[i]) | diag(g[i])));
      if (conflict || (!free_windows && g[i].kind == DK_J && g[j].kind == DK_J)) pred[size_t(j)].push_back(i);
    }
  std::vector<char> done(size_t(n), 0);
  auto ready = [&](int j) {
    for (int i : pred[size_t(j)])
      if (!done[size_t(i)]) return false;
    return true;
  };
  std::vector<RoundItem> out;
  int left = n;
  while (left > 0) {
    int i0 = 0;
    while (done[size_t(i0)] || !ready(i0)) ++i0;
    if (g[size_t(i0)].kind == DK_X || masked(g[size_t(i0)])) {
      out.push_back(RoundItem{i0, 0, 0});
      done[size_t(i0)] = 1;
      --left;
      continue;
    }
    uint32_t S = 0;
    std::vector<int> rnd;
    for (bool grew = true; grew;) {
      grew = false;
      for (int j = 0; j < n && !grew; ++j) {
        if (done[size_t(j)] || g[size_t(j)].kind == DK_X || masked(g[size_t(j)]) || !ready(j)) continue;
        const uint32_t m = mix(g[size_t(j)]);
        if (m && !(S & m) && __builtin_popcount(S) == kc) continue;
        S |= m;
        rnd.push_back(j);
        done[size_t(j)] = 1;
        --left;
        grew = true;
      }
    }
    if (S == 0) {  // E / Z only: each runs on its own
      for (int j : rnd) out.push_back(RoundItem{j, 0, 0});
      continue;
    }
    // fill the cube with the highest free bits: lanes then run over the low
    // bits, which keeps the LDS accesses of a cube free of bank conflicts
    for (int b = k - 1; __builtin_popcount(S) < kc && b >= 0; --b) S |= 1u << b;
    uint32_t bits = 0;
    int pos_of[32];
    for (int b = 0, i = 0; b < k; ++b)
      if (S & (1u << b)) {
        pos_of[b] = i;
        bits |= uint32_t(b) << (8 * i++);
      }
    // the round as sweeps: each applies its E / Z, then at most one window
    // per cube position in position order (a fixed code path per position);
    // every command goes to the first sweep after the commands it depends on
    struct Sweep {
      std::vector<int> diag;
      int win[4] = {-1, -1, -1, -1};
    };
    std::vector<Sweep> sweeps;
    std::vector<int> sweep_of(size_t(n), -1), slot_of(size_t(n), -2);  // slot -1: E / Z, else the position
    for (int j : rnd) {
      const bool win = g[size_t(j)].kind == DK_J;
      const int pj = win ? pos_of[g[size_t(j)].lb] : -1;
      int first = 0;
      for (int i : pred[size_t(j)]) {
        if (sweep_of[size_t(i)] < 0) continue;  // done in an earlier round
        const int si = sweep_of[size_t(i)], slot = slot_of[size_t(i)];
        const bool before = slot == -1 ? true : (win && slot < pj);  // runs earlier within the same sweep
        first = std::max(first, before ? si : si + 1);
      }
      int sw = first;
      if (win)
        while (sw < int(sweeps.size()) && sweeps[size_t(sw)].win[pj] >= 0) ++sw;
      if (sw >= int(sweeps.size())) sweeps.resize(size_t(sw) + 1);
      if (win) sweeps[size_t(sw)].win[pj] = j;
      else sweeps[size_t(sw)].diag.push_back(j);
      sweep_of[size_t(j)] = sw;
      slot_of[size_t(j)] = pj;
    }
    out.push_back(RoundItem{-1, int(rnd.size() + sweeps.size()), bits});
    for (const Sweep &w : sweeps) {
      uint32_t pm = 0;
      for (int p = 0; p < kc; ++p)
        if (w.win[p] >= 0) pm |= 1u << p;
      out.push_back(RoundItem{-2, int(w.diag.size()), pm});
      for (int j : w.diag) out.push_back(RoundItem{j, 0, 0});
      for (int p = 0; p < kc; ++p)
        if (w.win[p] >= 0) out.push_back(RoundItem{w.win[p], 0, 0});
    }
  }
  return out;
}

namespace {

// A window whose map is the same on every tile and in every order of the
// round: no local or outer masks, and p = 1/2 exactly (an odd E(v, w) count).
bool composable(const FuseOp &w) {
  return w.kind == DK_J && (w.lmask_b | w.lmask_o1) == 0 && (w.omask_b | w.omask_o1) == 0 && !(w.flags & 8u);
}

}  // namespace

// Windows on one position of a register round (one mixing bit) that follow
// each other with no E / Z on that bit between them commute with everything
// else between them (windows on other positions, E / Z on other bits), so
// the earlier ones may move up to the last one and the run is one linear
// map on the pair: the product of their 2x2 maps, formed in FP64 and rounded
// once to FP32.  It replaces the last window of the run (a DK_U row); the
// others leave their sweeps.  A DK_U costs the FP32 work of two windows.
// All or nothing: when every window of the group's rounds composes, each
// run (one window or more) becomes a map, so the kernel runs one code path
// per round position (maps only); otherwise nothing is composed.
bool merge_round_windows(const FuseOp *ops, int nops, int tile_bits, std::vector<FuseOp> &out,
                         std::vector<int> *src) {
  const int kc = tile_cube_bits(tile_bits);
  for (int q = 0; q < nops; ++q) {
    if (ops[q].kind != DK_R) continue;
    for (int o = q + 1; o <= q + ops[q].m_index; ++o)
      if (ops[o].kind == DK_J && !composable(ops[o])) return false;
    q += ops[q].m_index;
  }
  struct Sweep {
    FuseOp head;
    std::vector<FuseOp> diag;
    FuseOp win[4];
    bool has[4] = {false, false, false, false};
    int at[4] = {-1, -1, -1, -1};  // the window's row in ops
    std::vector<int> from[4];      // a map: the rows of its windows, in order
  };
  std::vector<FuseOp> res;
  std::vector<int> refs;
  res.reserve(size_t(nops));
  bool any = false;
  for (int q = 0; q < nops; ++q) {
    if (ops[q].kind != DK_R) {
      res.push_back(ops[q]);
      continue;
    }
    const FuseOp rh = ops[q];
    const int end = q + 1 + rh.m_index;
    std::vector<Sweep> sw;
    for (int o = q + 1; o < end;) {
      Sweep w;
      w.head = ops[o++];
      for (int d = 0; d < w.head.m_index; ++d) w.diag.push_back(ops[o++]);
      for (int pos = 0; pos < kc; ++pos)
        if ((w.head.flags >> pos) & 1u) {
          w.at[pos] = o;
          w.win[pos] = ops[o++];
          w.has[pos] = true;
        }
      sw.push_back(w);
    }
    q = end - 1;
    for (int pos = 0; pos < kc; ++pos) {
      const uint32_t bit = 1u << ((rh.lmask_b >> (8 * pos)) & 0xFFu);
      std::vector<size_t> run;
      auto flush = [&]() {
        if (!run.empty()) {
          double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
          std::vector<int> from;
          for (size_t i : run) {  // u <- W u, in the order the windows run
            double w[8];
            window_map(sw[i].win[pos], w);
            map_left(w, u);
            from.push_back(sw[i].at[pos]);
          }
          const FuseOp last = sw[run.back()].win[pos];
          FuseOp m{};
          m.kind = DK_U;
          m.lb = last.lb;
          m.widx = last.widx;
          m.m_index = last.m_index;
          map_store(m, u);
          for (size_t i = 0; i + 1 < run.size(); ++i) sw[run[i]].has[pos] = false;
          sw[run.back()].win[pos] = m;
          sw[run.back()].from[pos] = from;
          any = true;
        }
        run.clear();
      };
      for (size_t i = 0; i < sw.size(); ++i) {
        for (const FuseOp &d : sw[i].diag)
          if (d.lmask_b & bit) {  // an E / Z on this bit ends the run
            flush();
            break;
          }
        if (!sw[i].has[pos]) continue;
        run.push_back(i);  // every window of the rounds composes (checked above)
      }
      flush();
    }
    const size_t at = res.size();
    res.push_back(rh);
    for (const Sweep &w : sw) {
      uint32_t pm = 0;
      for (int pos = 0; pos < kc; ++pos)
        if (w.has[pos]) pm |= 1u << pos;
      if (pm == 0 && w.diag.empty()) continue;
      FuseOp h = w.head;
      h.flags = uint8_t(pm);
      res.push_back(h);
      for (const FuseOp &d : w.diag) res.push_back(d);
      for (int pos = 0; pos < kc; ++pos)
        if (w.has[pos]) {
          if (w.win[pos].kind == DK_U) {  // its row here, then its windows' rows in ops
            refs.push_back(int(res.size()));
            refs.push_back(int(w.from[pos].size()));
            refs.insert(refs.end(), w.from[pos].begin(), w.from[pos].end());
          }
          res.push_back(w.win[pos]);
        }
    }
    res[at].m_index = int(res.size() - at - 1);
  }
  if (!any) return false;
  out.swap(res);
  if (src) src->swap(refs);
  return true;
}

// Group runs of window/E/X/Z steps at one width >= kTileMinWidth into tile
// passes (see owqs_tile.hip).  A pass ends at N or M steps and at a width
// change; steps whose mixing slot would not fit the tile, or windows beyond
// the largest number one pass may chain (win_cap), are left for later passes
// while commuting steps after them still join.  The result goes to `out`: a step that joins no group is copied unchanged (all
// its fields), a group becomes one S_F step whose TileGroup is appended to
// `groups`, its commands to `fops` and its windows' measurement indices to
// `fm`.
void group_steps(const std::vector<Step> &steps, int mode, int tile_bits, std::vector<Step> &out,
                 std::vector<TileGroup> &groups, std::vector<FuseOp> &fops, std::vector<int> &fm, bool big_half,
                 std::vector<FuseOp> *mops, std::vector<int> *msrc) {
  const size_t ns = steps.size();
  // windows of a pass chain their norms in FP32 without renormalising: 16
  // keep it in range down to p ~ 1e-4 per window; windows with p = 1/2
  // exactly (an odd E(v, w) count) keep the norm, so a pass of only those
  // (and EOWQS, which computes no norm) may hold kMaxGroupWindows.  With
  // big_half (OWQS), a pass of only such windows runs without window sums
  // (mark_half makes it half, at most renormalising its output), so it may
  // hold kMaxHalfWindows.
  auto win_cap = [mode, big_half](bool even) {
    if (mode == OWQS_MODE_EOWQS) return kMaxGroupWindows;
    if (even) return 16;
    return big_half ? kMaxHalfWindows : kMaxGroupWindows;
  };
  auto groupable = [](int k) { return k == S_J || k == S_E || k == S_X || k == S_Z; };
  std::vector<char> done(ns, 0);
  std::vector<size_t> taken, skipped;
  size_t i = 0;
  while (true) {
    while (i < ns && done[i]) ++i;
    if (i == ns) break;
    const Step &x0 = steps[i];
    if (!groupable(x0.kind) || x0.n < kTileMinWidth) {
      out.push_back(x0);
      done[i] = 1;
      continue;
    }
    const int n = x0.n;
    int k = std::max(kMinTileBits, std::min(kDefaultTileBits, n - 8));
    if (tile_bits) k = std::min(tile_bits, n - 2);
    uint64_t tmask = (uint64_t(1) << kLowBits) - 1;
    int used = kLowBits, nwin = 0;
    bool even = false;  // the pass holds a window with an even E(v, w) count
    // Take the run's steps in order; a step that does not fit (its mixing
    // slot would overflow the tile, or the window count is reached) is left
    // for a later pass, and a later step may join only if it commutes with
    // every step left behind (commute_steps), up to kGroupLookahead steps.
    taken.clear();
    skipped.clear();
    for (size_t j = i; j < ns && j - i < kGroupLookahead; ++j) {
      if (done[j]) continue;
      const Step &x = steps[j];
      if (!groupable(x.kind) || x.n != n || taken.size() == 255) break;
      bool ok = !(x.kind == S_J && nwin >= win_cap(even || x.win.vw_even));
      uint64_t bit = 0;
      if (ok && (x.kind == S_J || x.kind == S_X)) {
        bit = uint64_t(1) << x.b0;
        if (tmask & bit) bit = 0;
        else if (used == k) ok = false;
      }
      for (size_t q = 0; ok && q < skipped.size(); ++q) ok = commute_steps(steps[skipped[q]], x);
      if (!ok) {
        skipped.push_back(j);
        if (skipped.size() > kGroupSkipMax) break;
        continue;
      }
      taken.push_back(j);
      if (bit) {
        tmask |= bit;
        ++used;
      }
      nwin += x.kind == S_J;
      even = even || (x.kind == S_J && x.win.vw_even);
    }
    if (taken.size() < 2) {
      out.push_back(x0);
      done[i] = 1;
      continue;
    }
    for (size_t q : taken) done[q] = 1;
    // fill the tile up to k bits with the lowest unused slots (more work per pass)
    for (int b = 0; used < k && b < n; ++b)
      if (!(tmask & (uint64_t(1) << b))) {
        tmask |= uint64_t(1) << b;
        ++used;
      }
    TileGroup tg{};
    tg.ta.n = n;
    tg.ta.k = k;
    tg.ta.tmask = tmask;
    tg.ta.omask = ((n >= 64 ? ~uint64_t(0) : (uint64_t(1) << n) - 1)) & ~tmask;
    int local_of[64];
    for (int b = 0, li = 0, oi = 0; b < n; ++b) {
      if (tmask & (uint64_t(1) << b)) {
        tg.ta.tpos[li] = (uint8_t)b;
        local_of[b] = li++;
      } else {
        tg.ta.opos[oi++] = (uint8_t)b;
        local_of[b] = -1;
      }
    }
    auto split = [&](uint64_t gmask, uint32_t &lm, uint64_t &om) {
      lm = 0;
      om = 0;
      for (int b = 0; b < n; ++b)
        if (gmask & (uint64_t(1) << b)) {
          if (local_of[b] >= 0) lm |= 1u << local_of[b];
          else om |= uint64_t(1) << b;
        }
    };
    tg.op_off = fops.size();
    tg.m_off = fm.size();
    std::vector<FuseOp> gops;
    for (size_t q : taken) {
      const Step &x = steps[q];
      FuseOp op{};
      op.kind = (uint8_t)x.kind;
      if (x.kind == S_J) {
        op.lb = (uint8_t)local_of[x.b0];
        op.flags = (x.win.swap ? 1 : 0) | (x.win.neg0 ? 2 : 0) | (x.win.neg1 ? 4 : 0) | (x.win.vw_even ? 8 : 0);
        op.m_index = x.m_index;
        op.f = (float)x.host_factor;
        // the factor times the coefficient (exact product of the two FP32 values, rounded once)
        op.coef = make_float2(float(double(op.f) * double(x.coef.x)), float(double(op.f) * double(x.coef.y)));
        split(x.win.mask_b, op.lmask_b, op.omask_b);
        split(x.win.mask_o1, op.lmask_o1, op.omask_o1);
        round_words(op);
      } else if (x.kind == S_X) {
        op.lb = (uint8_t)local_of[x.b0];
      } else if (x.kind == S_E) {
        split((uint64_t(1) << x.b0) | (uint64_t(1) << x.b1), op.lmask_b, op.omask_b);
      } else {  // S_Z
        split(uint64_t(1) << x.b0, op.lmask_b, op.omask_b);
      }
      gops.push_back(op);
    }
    // rounds over register cubes; windows keep their order where their
    // probabilities depend on it (a window with an even E(v, w) count)
    int widx = 0;
    for (const RoundItem &it : schedule_rounds(gops, k, !even)) {
      if (it.op == -1) {  // a round: its entries follow
        FuseOp h{};
        h.kind = DK_R;
        h.m_index = it.count;
        h.lmask_b = it.bits;
        fops.push_back(h);
        continue;
      }
      if (it.op == -2) {  // a sweep of the round: its E / Z, then its windows by position
        FuseOp h{};
        h.kind = DK_S;
        h.m_index = it.count;
        h.flags = uint8_t(it.bits);
        fops.push_back(h);
        continue;
      }
      FuseOp op = gops[size_t(it.op)];
      if (op.kind == S_J) {
        op.flags |= widx == 0 ? 16 : 0;  // the first window to run applies sigma
        op.widx = (uint8_t)widx++;
        fm.push_back(op.m_index);
      }
      fops.push_back(op);
    }
    tg.ta.nops = int(fops.size() - tg.op_off);
    tg.ta.nwin = widx;
    if (mops) {
      std::vector<FuseOp> m;
      std::vector<int> refs;
      if (merge_round_windows(fops.data() + tg.op_off, tg.ta.nops, k, m, &refs)) {
        tg.mop_off = mops->size();
        tg.mnops = int(m.size());
        mops->insert(mops->end(), m.begin(), m.end());
        if (msrc)  // each map: its row in mops, its window count, its windows' rows in fops
          for (size_t q = 0; q < refs.size();) {
            const int cnt = refs[q + 1];
            msrc->push_back(int(tg.mop_off) + refs[q]);
            msrc->push_back(cnt);
            for (int c = 0; c < cnt; ++c) msrc->push_back(int(tg.op_off) + refs[q + 2 + size_t(c)]);
            q += 2 + size_t(cnt);
          }
      }
    }
    tg.half = widx > 0 && !even;
    // compile the register runs in only where two windows on different bits
    // follow each other outside rounds, possibly with an E or Z between
    // (they cost occupancy elsewhere)
    tg.ta.runs = 0;
    {
      std::vector<const FuseOp *> top;  // the commands outside rounds, in order
      for (size_t q = tg.op_off; q < fops.size(); ++q) {
        if (fops[q].kind == DK_R) {
          top.push_back(nullptr);  // a round separates its neighbours
          q += size_t(fops[q].m_index);
          continue;
        }
        top.push_back(&fops[q]);
      }
      for (size_t q = 0; q + 1 < top.size(); ++q) {
        const FuseOp *a = top[q], *b = top[q + 1];
        if (!a || !b) continue;
        if (a->kind == S_J && b->kind == S_J && a->lb != b->lb) tg.ta.runs = 1;
        // a window, an E or Z, a window (the E / Z is applied between them)
        if (q + 2 < top.size() && top[q + 2] && a->kind == S_J && (b->kind == S_E || b->kind == S_Z) &&
            top[q + 2]->kind == S_J && top[q + 2]->lb != a->lb)
          tg.ta.runs = 1;
      }
    }
    Step gs{};
    gs.kind = S_F;
    gs.n = n;
    gs.group = (int)groups.size();
    groups.push_back(tg);
    out.push_back(gs);
  }
}

void group_tiles(owqs_pattern *p) {
  p->xsteps.clear();
  p->groups.clear();
  p->fuse_ops.clear();
  p->fuse_m.clear();
  p->fuse_mops.clear();
  p->fuse_msrc.clear();
  if (p->exec == OWQS_EXEC_PLAIN) {
    p->xsteps = p->steps;
    return;
  }
  group_steps(p->steps, p->mode, p->tile_bits, p->xsteps, p->groups, p->fuse_ops, p->fuse_m,
              p->mode == OWQS_MODE_OWQS && p->half_cap > 0, &p->fuse_mops, &p->fuse_msrc);
  if (p->mode == OWQS_MODE_OWQS) mark_half(p->xsteps, p->groups, p->half_cap);
  else
    for (TileGroup &tg : p->groups) tg.half = false;
}

// State after each command of a plain plan (for ranged runs).
struct PlanTrace {
  std::vector<size_t> &step_end;
  std::vector<int> &width;
  std::vector<double> &pending;
  std::vector<int> &qubits;
};

// Translate the command list into steps (Sec. 4.4: N appends the top slot,
// M moves the top qubit into the measured slot); with `fused`, runs of the
// form N w; E's; M v; X/Z on w become one window step.
void compile_plan(owqs_pattern *p, bool fused, std::vector<Step> &steps, std::vector<int> &final_where,
                  double &final_factor, PlanTrace *tr) {
  const int nq = p->nq;
  std::vector<int> slot_of(nq, -1), qubit_at(OWQS_MAX_WIDTH + 1, -1), outcome_of(nq, 0);
  int n = (int)p->inputs.size();
  for (int k = 0; k < n; ++k) {
    slot_of[p->inputs[k]] = k;
    qubit_at[k] = p->inputs[k];
  }
  const double r2 = 1.0 / std::sqrt(2.0);
  double pending = 1.0;
  int m = 0;
  steps.clear();
  const size_t nc = p->cmds.size();
  if (tr) {
    tr->step_end.assign(nc, 0);
    tr->width.assign(nc, 0);
    tr->pending.assign(nc, 1.0);
    tr->qubits.assign(nc * kTraceStride, -1);
  }

  int last_s = 0, last_t = 0;
  auto coef_of = [&](const Cmd &c, int mi, int &o_out) {
    const int s = signal(c.s, outcome_of), t = signal(c.t, outcome_of);
    last_s = s;
    last_t = t;
    const double theta = (s ? -p->angles[mi] : p->angles[mi]) + (t ? M_PI : 0.0);  // Eq. 2
    const int o = p->outcomes[mi] & 1;
    double cr = std::cos(theta), ci = -std::sin(theta);  // e^{-i theta}  (Eqs. 11-12)
    if (o) { cr = -cr; ci = -ci; }
    o_out = o;
    return make_float2((float)cr, (float)ci);
  };

  for (size_t i = 0; i < nc; ++i) {
    const Cmd &c = p->cmds[i];
    // Window N w; E ... (each on v or w); M v; then X/Z on w, as one
    // in-place 2x2 pass over v's slot (E's to other qubits become signs).
    if (fused && c.op == OWQS_OP_N && i + 2 < nc) {
      const int w = c.q0;
      size_t j = i + 1;
      while (j < nc && p->cmds[j].op == OWQS_OP_E) ++j;
      if (j > i + 1 && j < nc && p->cmds[j].op == OWQS_OP_M && p->cmds[j].q0 != w) {
        const Cmd &mm = p->cmds[j];
        const int v = mm.q0;
        bool ok = slot_of[v] >= 0;
        int vw = 0;
        uint64_t mask_b = 0, mask_o1 = 0;
        for (size_t k = i + 1; k < j && ok; ++k) {
          const int a = p->cmds[k].q0, b = p->cmds[k].q1;
          if ((a == v && b == w) || (a == w && b == v)) {
            ++vw;
          } else if (a == v || b == v) {
            const int x = a == v ? b : a;
            ok = slot_of[x] >= 0;
            if (ok) mask_b ^= uint64_t(1) << slot_of[x];
          } else if (a == w || b == w) {
            const int y = a == w ? b : a;
            ok = slot_of[y] >= 0;
            if (ok) mask_o1 ^= uint64_t(1) << slot_of[y];
          } else {
            ok = false;  // an E on two other qubits ends the window
          }
        }
        if (ok && vw > 0) {
          int o = 0;
          Step st{};
          st.kind = S_J;
          st.n = n;
          st.b0 = slot_of[v];
          st.coef = coef_of(mm, m, o);
          st.sig_s = last_s;
          st.sig_t = last_t;
          st.outcome = o;
          st.host_factor = pending * r2;
          st.m_index = m;
          outcome_of[v] = o;
          ++m;
          st.win.mask_b = mask_b;
          st.win.mask_o1 = mask_o1;
          st.win.vw_even = (vw % 2 == 0) ? 1 : 0;
          // fold the following corrections on w into a signed permutation
          int idx[2] = {0, 1}, sgn[2] = {1, 1};
          size_t k = j + 1;
          while (k < nc && (p->cmds[k].op == OWQS_OP_X || p->cmds[k].op == OWQS_OP_Z) && p->cmds[k].q0 == w) {
            if (signal(p->cmds[k].s, outcome_of)) {
              if (p->cmds[k].op == OWQS_OP_X) {
                std::swap(idx[0], idx[1]);
                std::swap(sgn[0], sgn[1]);
              } else {
                sgn[1] = -sgn[1];
              }
            }
            ++k;
          }
          st.win.swap = idx[0] == 1;
          st.win.neg0 = sgn[0] < 0;
          st.win.neg1 = sgn[1] < 0;
          steps.push_back(st);
          slot_of[w] = st.b0;
          qubit_at[st.b0] = w;
          slot_of[v] = -1;
          pending = 1.0;
          i = k - 1;
          continue;
        }
      }
    }
    switch (c.op) {
      case OWQS_OP_N: {
        Step st{};
        st.kind = S_N;
        st.n = n;
        steps.push_back(st);
        slot_of[c.q0] = n;
        qubit_at[n] = c.q0;
        ++n;
        pending *= r2;
        break;
      }
      case OWQS_OP_E: {
        Step st{};
        st.kind = S_E;
        st.n = n;
        st.b0 = slot_of[c.q0];
        st.b1 = slot_of[c.q1];
        steps.push_back(st);
        break;
      }
      case OWQS_OP_X:
      case OWQS_OP_Z: {
        if (signal(c.s, outcome_of)) {
          Step st{};
          st.kind = c.op == OWQS_OP_X ? S_X : S_Z;
          st.n = n;
          st.b0 = slot_of[c.q0];
          steps.push_back(st);
        }
        break;
      }
      case OWQS_OP_M: {
        int o = 0;
        Step st{};
        st.kind = S_M;
        st.n = n;
        st.b0 = slot_of[c.q0];
        st.coef = coef_of(c, m, o);
        st.sig_s = last_s;
        st.sig_t = last_t;
        st.outcome = o;
        st.host_factor = pending;
        st.m_index = m;
        steps.push_back(st);
        outcome_of[c.q0] = o;
        ++m;
        const int t = n - 1;
        if (st.b0 != t) {
          const int top = qubit_at[t];
          slot_of[top] = st.b0;
          qubit_at[st.b0] = top;
        }
        qubit_at[t] = -1;
        slot_of[c.q0] = -1;
        --n;
        pending = 1.0;
        break;
      }
      default:
        break;
    }
    if (tr) {
      tr->step_end[i] = steps.size();
      tr->width[i] = n;
      tr->pending[i] = pending;
      for (int b = 0; b < n; ++b) tr->qubits[i * kTraceStride + b] = qubit_at[b];
    }
  }
  final_where.assign(p->outputs.size(), 0);
  for (size_t k = 0; k < p->outputs.size(); ++k) final_where[k] = slot_of[p->outputs[k]];
  final_factor = pending;
}

// Compile the command list into device steps for the current settings.
void compile(owqs_pattern *p) {
  if (p->exec == OWQS_EXEC_SUBSTATES) {
    compile_substates(p);
    drop_ss_graph(p);
    p->plan_width = std::max(p->ss_width, 1);
    p->dirty = false;
    return;
  }
  compile_plan(p, p->exec != OWQS_EXEC_PLAIN, p->steps, p->final_where, p->final_factor, nullptr);
  if (p->mode == OWQS_MODE_OWQS) {  // windows with p = 1/2 do not renormalise (half_prob)
    double e = 1.0;
    for (Step &x : p->steps) {
      if (x.kind == S_J && !x.win.vw_even) x.host_factor = rounded_factor(x.host_factor, e);
      else if (x.kind == S_M || x.kind == S_J) e = 1.0;
    }
  }
  p->lk_valid = false;
  p->lk_next = SIZE_MAX;
  int w = std::max<int>((int)p->inputs.size(), (int)p->outputs.size());
  for (const Step &x : p->steps) w = std::max(w, x.n + (x.kind == S_N ? 1 : 0));
  p->plan_width = std::max(w, 1);
  group_tiles(p);
  static std::atomic<uint64_t> generation{0};
  p->plan_gen = ++generation;
  p->dirty = false;
  p->dev_steps_valid = false;
  p->dev_fuse_valid = false;
  if (p->graph_exec || p->graph || p->a_exec) (void)hipDeviceSynchronize();  // a replay may still be in flight
  if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
  if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
  if (p->a_exec) { (void)hipGraphExecDestroy(p->a_exec); p->a_exec = nullptr; }
  if (p->a_graph) { (void)hipGraphDestroy(p->a_graph); p->a_graph = nullptr; }
}

// Patterns of any width load (so they can be reordered and read back); only
// those within OWQS_MAX_WIDTH compile and run.
void compile(owqs_pattern *p);

owqs_status width_guard(owqs_pattern *p) {
  if (p->exec == OWQS_EXEC_SUBSTATES) {
    if (p->dirty) compile(p);
    if (p->ss_width > OWQS_MAX_WIDTH)
      return fail(p->ctx, OWQS_E_WIDTH, "sub-state width " + std::to_string(p->ss_width) + " above OWQS_MAX_WIDTH");
    if (!p->ss_plan_ok) return fail(p->ctx, OWQS_E_STATE, "internal error: a sub-state step outside its region");
    return OWQS_OK;
  }
  if (p->max_live > OWQS_MAX_WIDTH)
    return fail(p->ctx, OWQS_E_WIDTH, "live width " + std::to_string(p->max_live) +
                                          " above OWQS_MAX_WIDTH (owqs_pattern_reorder can narrow it)");
  return OWQS_OK;
}

owqs_status ensure_device(owqs_pattern *p, bool need_psi) {
  if (owqs_status w = width_guard(p)) return w;
  if (p->ctx->device < 0) return fail(p->ctx, OWQS_E_STATE, "host-only context (device -1) cannot run patterns");
  hipError_t e = hipSetDevice(p->ctx->device);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "hipSetDevice");
  // max_live may exceed the width limit (and 63) for sub-state patterns,
  // which never ask for the one-vector buffer
  if (need_psi && p->max_live > OWQS_MAX_WIDTH) return fail(p->ctx, OWQS_E_WIDTH, "live width over the limit");
  const size_t need = need_psi ? std::max<size_t>(size_t(1) << p->max_live, 4) : 0;
  if (need_psi && p->psi_cap < need) {
    if (p->psi) (void)hipFree(p->psi);
    p->psi = nullptr;
    p->psi_cap = 0;
    e = hipMalloc(&p->psi, need * sizeof(float2));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, std::string("state buffer: ") + hipGetErrorString(e));
    p->psi_cap = need;
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    if (p->a_exec) { (void)hipGraphExecDestroy(p->a_exec); p->a_exec = nullptr; }
    if (p->a_graph) { (void)hipGraphDestroy(p->a_graph); p->a_graph = nullptr; }
  }
  if (!p->book_mem) {
    const size_t nprob = std::max(p->n_meas, 1);
    const size_t bytes = 64 + nprob * sizeof(double) + kMaxPartials * sizeof(double) + 64;
    e = hipMalloc(&p->book_mem, bytes);
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, std::string("bookkeeping: ") + hipGetErrorString(e));
    char *b = static_cast<char *>(p->book_mem);
    p->book.sigma = reinterpret_cast<double *>(b);
    p->book.err = reinterpret_cast<int *>(b + 16);
    p->book.partials = reinterpret_cast<double *>(b + 64);
    p->book.probs = reinterpret_cast<double *>(b + 64 + kMaxPartials * sizeof(double));
  }
  return OWQS_OK;
}

owqs_status build_pattern(owqs_ctx *ctx, const owqs_cmd *cmds, size_t ncmds, const int32_t *dom, size_t ndom,
                          const int32_t *inputs, int32_t nin, const int32_t *outputs, int32_t nout,
                          owqs_pattern **out) {
  if (!ctx || !out || (ncmds && !cmds) || (ndom && !dom) || nin < 0 || nout < 0 || (nin && !inputs) ||
      (nout && !outputs))
    return fail(ctx, OWQS_E_INVALID_ARG, "null pointer or negative size");
  auto *p = new owqs_pattern();
  p->ctx = ctx;
  std::unordered_map<int32_t, int> dense;
  auto id = [&](int32_t q) -> int {
    auto it = dense.find(q);
    if (it != dense.end()) return it->second;
    const int d = (int)dense.size();
    dense.emplace(q, d);
    return d;
  };
  for (int k = 0; k < nin; ++k) {
    if (inputs[k] < 0) { delete p; return fail(ctx, OWQS_E_INVALID_ARG, "negative qubit id"); }
    p->inputs.push_back(id(inputs[k]));
  }
  for (int k = 0; k < nout; ++k) {
    if (outputs[k] < 0) { delete p; return fail(ctx, OWQS_E_INVALID_ARG, "negative qubit id"); }
    p->outputs.push_back(id(outputs[k]));
  }
  auto domain = [&](int32_t off, int32_t len, std::vector<int> &d) -> bool {
    if (len == 0) return true;
    if (off < 0 || len < 0 || size_t(off) + size_t(len) > ndom) return false;
    for (int32_t k = 0; k < len; ++k) {
      if (dom[off + k] < 0) return false;
      d.push_back(id(dom[off + k]));
    }
    return true;
  };
  for (size_t i = 0; i < ncmds; ++i) {
    const owqs_cmd &c = cmds[i];
    Cmd d{};
    d.op = c.op;
    if (c.op < OWQS_OP_N || c.op > OWQS_OP_Z || c.q0 < 0 || (c.op == OWQS_OP_E && c.q1 < 0)) {
      delete p;
      return fail(ctx, OWQS_E_INVALID_ARG, "command " + std::to_string(i) + ": bad opcode or qubit id");
    }
    d.q0 = id(c.q0);
    d.q1 = c.op == OWQS_OP_E ? id(c.q1) : -1;
    d.angle = c.angle;
    const bool has_s = c.op == OWQS_OP_M || c.op == OWQS_OP_X || c.op == OWQS_OP_Z;
    if (has_s && !domain(c.s_off, c.s_len, d.s)) {
      delete p;
      return fail(ctx, OWQS_E_INVALID_ARG, "command " + std::to_string(i) + ": bad s-domain range");
    }
    if (c.op == OWQS_OP_M && !domain(c.t_off, c.t_len, d.t)) {
      delete p;
      return fail(ctx, OWQS_E_INVALID_ARG, "command " + std::to_string(i) + ": bad t-domain range");
    }
    p->cmds.push_back(std::move(d));
  }
  p->nq = (int)dense.size();
  p->user_id.assign(p->nq, -1);
  for (const auto &kv : dense) p->user_id[kv.second] = kv.first;
  owqs_status st = validate(p);
  if (st != OWQS_OK) {
    delete p;
    return st;
  }
  for (const Cmd &c : p->cmds)
    if (c.op == OWQS_OP_M) p->angles.push_back(c.angle);
  p->outcomes.assign(p->n_meas, 0);
  *out = p;
  return OWQS_OK;
}

// Algorithmic bytes of one step (element level, complex64).
// Algorithmic bytes of a step at line granularity (a 128-byte line holds the
// 16 amplitudes of slots 0..3): E reads and writes the |11> quarter, or the
// half of the lines with the high bit set when the low bit is below 4, or
// every line when both are; Z the same for its one bit.
double step_bytes(const Step &x) {
  const double a = std::ldexp(8.0, x.n);  // 8 bytes * 2^n
  switch (x.kind) {
    case S_N: return 2.0 * a;
    case S_E: {
      const int lo = std::min(x.b0, x.b1), hi = std::max(x.b0, x.b1);
      return hi < 4 ? 2.0 * a : lo < 4 ? 1.0 * a : 0.5 * a;
    }
    case S_M: return 1.5 * a;
    case S_X: return 2.0 * a;
    case S_Z: return x.b0 < 4 ? 2.0 * a : 1.0 * a;
    case S_J: return 2.0 * a;
    case S_F: return 2.0 * a;  // one read and one write of the vector
  }
  return 0.0;
}

// Enqueue every step of the plan on `s`; with `ev`, record events around the
// main kernel and the finishing kernel of each step (see run_impl).
int *fuse_m_dev(owqs_pattern *p) { return reinterpret_cast<int *>(p->dev_fuse + p->fuse_ops.size()); }

// A window whose fresh qubit w meets v through an odd number of E has outcome
// probability exactly 1/2 for every state (Eqs. 11-13: the two outputs are
// f (a + t) and +-f (a - t) with |t| = f |b|, so their squared norms add up
// to 2 f^2 (|a|^2 + |b|^2) whatever the coefficient).  In OWQS mode such a
// window needs no reduction: p = 1/2 is recorded, and since the pass then
// keeps the norm of its input, sigma is left for the next measurement.
bool half_prob(const Step &x, int reduce) { return reduce == kReduceRenorm && x.kind == S_J && x.half; }

// Such windows scale the vector by their factor rounded to FP32, and no
// reduction renormalises it after them, so the rounding would compound (for
// 1/sqrt 2, by 3.4e-8 in |psi|^2 per window).  The factors are chosen in
// execution order with error feedback instead: `e` is the ratio of the
// vector's scale to the exact one so far; the next factor aims at h / e and
// e takes up what its FP32 rounding leaves, so |e - 1| stays within one
// rounding.  Returns the factor to use (its FP32 rounding is what the
// kernels apply).
double rounded_factor(double h, double &e) {
  const double t = h / e;
  e *= double(float(t)) / h;
  return t;
}

// What the FP32 arithmetic of a window leaves in |psi|^2 beyond its factor
// (the rounding of the coefficient, at most a few 1e-8 per window) would
// still add up over a long run without reductions, so at most cap such
// windows pass between two renormalisations.  When the next window or group
// would exceed cap, the last tile group of the run so far sums the norm of
// its output (renorm: sigma is reset from it, its windows still record
// p = 1/2 without sums) and the run restarts after it; with no such group
// to take it, a single window reduces as usual and a group renormalises its
// own output.  cap = 0: every window and group reduces.
void mark_half(std::vector<Step> &xs, std::vector<TileGroup> &groups, int cap) {
  int run = 0;     // windows with p = 1/2 since the last renormalisation
  int last = -1;   // the run's last half group, which may still take the renormalisation
  int after = 0;   // windows of the run after that group
  auto restart = [&] {
    run = 0;
    last = -1;
    after = 0;
  };
  auto make_room = [&](int need) {
    if (run + need > cap && last >= 0) {
      groups[size_t(last)].renorm = true;
      run = after;
      last = -1;
      after = 0;
    }
  };
  for (TileGroup &tg : groups) tg.renorm = false;
  for (Step &x : xs) {
    if (x.kind == S_M) {
      restart();
    } else if (x.kind == S_J) {
      if (!x.win.vw_even) make_room(1);
      x.half = !x.win.vw_even && run + 1 <= cap;
      if (x.half) {
        ++run;
        ++after;
      } else {
        restart();
      }
    } else if (x.kind == S_F) {
      TileGroup &tg = groups[x.group];
      if (tg.ta.nwin == 0) continue;  // no norm changes, no reduction
      tg.half = tg.half && cap > 0;
      if (!tg.half) {
        restart();
        continue;
      }
      make_room(tg.ta.nwin);
      if (run + tg.ta.nwin > cap) {
        tg.renorm = true;
        restart();
      } else {
        run += tg.ta.nwin;
        last = x.group;
        after = 0;
      }
    }
  }
}

hipError_t launch_range(owqs_pattern *p, const std::vector<Step> &xs, size_t i0, size_t i1, int reduce,
                        hipStream_t s, std::vector<hipEvent_t> *ev, const float2 *ctab, const int *ftab,
                        float2 *psi_over, const DevBook *book_over, bool groups_patched) {
  float2 *const psi = psi_over ? psi_over : p->psi;
  const DevBook book = book_over ? *book_over : p->book;
  hipError_t e = hipSuccess;
  for (size_t i = i0; i < i1 && e == hipSuccess; ++i) {
    const Step &x = xs[i];
    MeasureArgs a{};
    a.reduce = reduce;
    a.book = book;
    unsigned grid = 0;
    const FuseOp *ops = nullptr;
    switch (x.kind) {
      case S_N: e = launch_prepare(psi, x.n, s); break;
      case S_E: e = launch_cz(psi, x.n, x.b0, x.b1, s); break;
      case S_X: e = launch_pauli_x(psi, x.n, x.b0, s); break;
      case S_Z: e = launch_pauli_z(psi, x.n, x.b0, s); break;
      case S_M:
      case S_J:
        a.coef = x.coef;
        a.host_factor = x.host_factor;
        a.m_index = x.m_index;
        if (half_prob(x, reduce)) {  // p = 1/2 exactly: no reduction, sigma carried to the next M
          a.reduce = kReduceNone;
          a.prob_half = 1;
        }
        if (ctab && x.kind == S_J) {
          a.coef_dev = ctab + x.m_index;
          a.fold_dev = ftab + 3 * x.m_index;
        }
        e = x.kind == S_M ? launch_measure(psi, x.n, x.b0, a, s, &grid)
                          : launch_jwindow(psi, x.n, x.b0, a, x.win, s, &grid);
        break;
      case S_F: {
        const TileGroup &tg = p->groups[x.group];
        ops = p->dev_fuse + tg.op_off;
        TileArgs ta = tg.ta;
        if (ctab && !groups_patched) {
          ta.coefs = ctab;
          ta.nsets = 1;
          ta.folds = ftab;
        }
        if (reduce == kReduceRenorm && tg.half) {  // every window has p = 1/2 exactly
          a.reduce = kReduceNone;
          ta.half_m = fuse_m_dev(p) + tg.m_off;
          ta.renorm = tg.renorm ? 1 : 0;
        }
        // no window sums: the composed commands (a drawn run that patches the
        // rows has composed them again on the device, k_s_compose)
        if (tg.mnops > 0 && (!ctab || groups_patched) && a.reduce == kReduceNone) {
          ops = p->dev_fuse + fuse_mops_base(p->fuse_ops.size(), p->fuse_m.size()) + tg.mop_off;
          ta.nops = tg.mnops;
          ta.maps = 1;
        }
        e = launch_tile(psi, ta, ops, a, s, &grid);
        break;
      }
      default: break;
    }
    if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 1], s);
    if ((x.kind == S_M || x.kind == S_J) && e == hipSuccess) e = launch_finish(a, grid, s);
    if (x.kind == S_F && e == hipSuccess) {
      const TileGroup &tg = p->groups[x.group];
      if (reduce == kReduceRenorm && tg.half && tg.renorm) e = launch_finish_renorm(a.book, grid, s);
      else e = launch_finish_group(a, fuse_m_dev(p) + tg.m_off, tg.ta.nwin, grid, s);
    }
    if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 2], s);
  }
  return e;
}

hipError_t launch_steps(owqs_pattern *p, int reduce, hipStream_t s, std::vector<hipEvent_t> *ev) {
  return launch_range(p, p->xsteps, 0, p->xsteps.size(), reduce, s, ev);
}

// Upload the tile groups' command table: FuseOps, then the windows'
// measurement indices.
size_t fuse_mops_base(size_t nfops, size_t nfm) {
  return nfops + (nfm * sizeof(int) + sizeof(FuseOp) - 1) / sizeof(FuseOp);
}

owqs_status upload_fuse_table(owqs_ctx *ctx, const std::vector<FuseOp> &fops, const std::vector<int> &fm,
                              FuseOp *&dev, size_t &cap, const std::vector<FuseOp> *mops) {
  static const hipError_t prep = tile_prepare();  // once per process, outside any capture
  if (prep != hipSuccess) return hip_fail(ctx, prep, "tile kernel attribute");
  const size_t base = fuse_mops_base(fops.size(), fm.size());
  const size_t nm = mops ? mops->size() : 0;
  const size_t need = std::max<size_t>(base + nm, 1);
  hipError_t e = hipSuccess;
  if (dev) (void)hipDeviceSynchronize();  // a run in flight may still read the old table
  if (cap < need) {
    if (dev) (void)hipFree(dev);
    dev = nullptr;
    cap = 0;
    e = hipMalloc(&dev, need * sizeof(FuseOp));
    if (e != hipSuccess) return fail(ctx, OWQS_E_NOMEM, "fused command table");
    cap = need;
  }
  if (!fops.empty()) e = hipMemcpy(dev, fops.data(), fops.size() * sizeof(FuseOp), hipMemcpyHostToDevice);
  if (e == hipSuccess && !fm.empty())
    e = hipMemcpy(reinterpret_cast<int *>(dev + fops.size()), fm.data(), fm.size() * sizeof(int),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && nm) e = hipMemcpy(dev + base, mops->data(), nm * sizeof(FuseOp), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "fused command table upload");
  return OWQS_OK;
}

owqs_status upload_fuse(owqs_pattern *p) {
  if (p->dev_fuse_valid && !p->fuse_patched) return OWQS_OK;
  const owqs_status st =
      upload_fuse_table(p->ctx, p->fuse_ops, p->fuse_m, p->dev_fuse, p->dev_fuse_cap, &p->fuse_mops);
  if (st == OWQS_OK) {
    p->dev_fuse_valid = true;
    p->fuse_patched = false;
  }
  return st;
}

// Upload the plan as a DevStep table (for the LDS-resident kernels).
namespace {

// A window step's map as the LDS-resident kernel applies it without masks
// and without renormalising (EOWQS): o0 = f (a + c b), o1 = f (a + s1 c b)
// with s1 = +1 for an even E(v, w) count, then the folded exchange and
// negations (run_item in owqs_batch.hip).  Row-major, (re, im) pairs.
void lds_window_map(const DevStep &st, double m[8]) {
  const double f = st.host_factor, cx = st.coef.x, cy = st.coef.y, s1 = (st.pp & 8u) ? 1.0 : -1.0;
  double r0[4] = {f, 0.0, f * cx, f * cy}, r1[4] = {f, 0.0, s1 * f * cx, s1 * f * cy};
  if (st.pp & 1u)
    for (int k = 0; k < 4; ++k) {
      const double t = r0[k];
      r0[k] = r1[k];
      r1[k] = t;
    }
  const double n0 = (st.pp & 2u) ? -1.0 : 1.0, n1 = (st.pp & 4u) ? -1.0 : 1.0;
  for (int k = 0; k < 4; ++k) {
    m[k] = n0 * r0[k];
    m[4 + k] = n1 * r1[k];
  }
}

// Compose runs of unmasked window steps on one slot (LDS tables): a window
// joins the last window on its slot when no step since then touched that
// slot (E, X or Z on it, a window reading it as a sign) and no N or M
// changed the layout; the steps between commute with the earlier windows,
// so they may move down to the latest one, whose row becomes their product
// (DK_U, entries as FP32 words: m00 in coef, m01 in host_factor and pp, m10
// and m11 in mask_b and mask_o1, low word re, high word im).  Rows move
// later, never earlier, so no window meets more windows recorded without a
// sum before it than it did.
// With `owqs` (OWQS, the kernel renormalising), only windows that run_item
// records with p = 1/2 and no sum compose (an odd E(v, w) count, fewer than
// kHalfRun such windows since the last sum, found by replaying its rule), a
// window or M that sums ends every run, and a composed row lists its
// windows' measurement indices in `mlist` (m_index: the first, b1: the
// count), for which the kernel records 1/2.
std::vector<DevStep> compose_lds_steps(const std::vector<DevStep> &d, bool owqs, std::vector<int> &mlist) {
  std::vector<DevStep> out;
  std::vector<std::array<double, 8>> prod;  // the product of each composed row so far
  std::vector<std::vector<int>> ms;         // the measurement indices of each row's windows
  std::vector<char> dead;                   // rows whose windows moved down into a later row
  std::vector<int> open(64, -1);            // per slot: the row of its open run
  int half_run = 0;
  for (const DevStep &st : d) {
    bool win = st.kind == DK_J;
    const bool masked = win && (st.mask_b | st.mask_o1) != 0;
    bool sums = st.kind == DK_M;
    if (owqs && win) {
      const bool half = !(st.pp & 24u) && half_run < kHalfRun;
      if (half) ++half_run;
      else sums = true;
    }
    if (owqs && sums) half_run = 0;
    if (st.kind == DK_N || st.kind == DK_M || (owqs && sums)) {
      std::fill(open.begin(), open.end(), -1);
      if (sums) win = false;  // a window that sums stays as it is
    } else if (st.kind == DK_E) {
      open[st.b0] = open[st.b1] = -1;
    } else if (st.kind == DK_X || st.kind == DK_Z) {
      open[st.b0] = -1;
    } else if (masked) {
      for (int b = 0; b < 64; ++b)
        if (((st.mask_b | st.mask_o1) >> b) & 1u) open[b] = -1;
      open[st.b0] = -1;
    }
    if (win && !masked && open[st.b0] >= 0) {  // joins the run on its slot, in its own place
      const size_t r = size_t(open[st.b0]);
      double w[8];
      lds_window_map(st, w);
      std::array<double, 8> u = prod[r];
      map_left(w, u.data());
      std::vector<int> m = std::move(ms[r]);
      m.push_back(st.m_index);
      dead[r] = 1;
      DevStep row = st;
      row.kind = DK_U;
      out.push_back(row);
      prod.push_back(u);
      ms.push_back(std::move(m));
      dead.push_back(0);
      open[st.b0] = ms.back().size() < 255 ? int(out.size() - 1) : -1;
      continue;
    }
    out.push_back(st);
    prod.emplace_back();
    ms.emplace_back(1, st.m_index);
    dead.push_back(0);
    if (win && !masked) {
      lds_window_map(st, prod.back().data());
      open[st.b0] = int(out.size() - 1);
    }
  }
  std::vector<DevStep> kept;
  for (size_t r = 0; r < out.size(); ++r) {
    if (dead[r]) continue;
    kept.push_back(out[r]);
    if (out[r].kind != DK_U) continue;
    DevStep &k = kept.back();
    k.m_index = int(mlist.size());
    k.b1 = uint8_t(ms[r].size());
    mlist.insert(mlist.end(), ms[r].begin(), ms[r].end());
    float f[8];
    for (int q = 0; q < 8; ++q) f[q] = float(prod[r][size_t(q)]);
    uint32_t w[8];
    __builtin_memcpy(w, f, sizeof(w));
    k.coef = make_float2(f[0], f[1]);
    k.host_factor = f[2];
    k.pp = w[3];
    k.mask_b = uint64_t(w[4]) | (uint64_t(w[5]) << 32);
    k.mask_o1 = uint64_t(w[6]) | (uint64_t(w[7]) << 32);
  }
  return kept;
}

}  // namespace

owqs_status upload_steps(owqs_pattern *p) {
  if (p->dev_steps_valid) return OWQS_OK;
  std::vector<DevStep> d(p->steps.size());
  for (size_t i = 0; i < d.size(); ++i) {
    const Step &x = p->steps[i];
    d[i].kind = (uint8_t)x.kind;
    d[i].n = (uint8_t)x.n;
    d[i].b0 = (uint8_t)x.b0;
    d[i].b1 = (uint8_t)x.b1;
    d[i].m_index = x.m_index;
    d[i].coef = x.coef;
    d[i].host_factor = (float)x.host_factor;
    d[i].pp = (x.win.swap ? 1u : 0u) | (x.win.neg0 ? 2u : 0u) | (x.win.neg1 ? 4u : 0u) | (x.win.vw_even ? 8u : 0u) |
              (p->half_cap == 0 ? 16u : 0u);
    d[i].mask_b = x.win.mask_b;
    d[i].mask_o1 = x.win.mask_o1;
  }
  // runs of windows on one slot compose where no window of the run sums
  // (EOWQS; OWQS windows recorded with p = 1/2), at most 255 to a row
  std::vector<int> mlist;
  const int red = reduce_of(p);
  if (red == kReduceNone || red == kReduceRenorm) d = compose_lds_steps(d, red == kReduceRenorm, mlist);
  p->dev_nsteps = d.size();
  // the composed rows' measurement indices follow the rows
  const size_t need = std::max<size_t>(d.size() + (mlist.size() * sizeof(int) + sizeof(DevStep) - 1) / sizeof(DevStep), 1);
  hipError_t e = hipSuccess;
  if (p->dev_steps_cap < need) {
    if (p->dev_steps) (void)hipFree(p->dev_steps);
    p->dev_steps = nullptr;
    p->dev_steps_cap = 0;
    e = hipMalloc(&p->dev_steps, need * sizeof(DevStep));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "command table");
    p->dev_steps_cap = need;
  }
  if (!d.empty()) e = hipMemcpy(p->dev_steps, d.data(), d.size() * sizeof(DevStep), hipMemcpyHostToDevice);
  if (e == hipSuccess && !mlist.empty())
    e = hipMemcpy(reinterpret_cast<int *>(p->dev_steps + d.size()), mlist.data(), mlist.size() * sizeof(int),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "command table upload");
  p->dev_steps_valid = true;
  return OWQS_OK;
}

int reduce_of(const owqs_pattern *p) {
  return p->mode == OWQS_MODE_OWQS ? kReduceRenorm : p->mode == OWQS_MODE_EOWQS_CHECK ? kReduceCheck : kReduceNone;
}

LdsItem lds_proto(const owqs_pattern *p) {
  LdsItem it{};
  it.steps = p->dev_steps;
  it.nsteps = (int)p->dev_nsteps;
  it.nin = (int)p->inputs.size();
  it.nout = (int)p->outputs.size();
  it.final_factor = p->final_factor;
  it.basis = -1;
  for (size_t k = 0; k < p->final_where.size(); ++k) it.where[k] = p->final_where[k];
  return it;
}

// Any other run overwrites the state (or its scale) that a ranged run left.
void end_ranged(owqs_pattern *p) {
  p->lk_next = SIZE_MAX;
  p->lk_ran = false;
}

owqs_status run_impl(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device, void *stream,
                     Profile *prof) {
  if (p && substates(p)) {
    const size_t nin = p->inputs.size();
    if (nin > OWQS_MAX_WIDTH) return fail(p->ctx, OWQS_E_WIDTH, "more inputs than OWQS_MAX_WIDTH: give them as factors");
    if (n_amps != (size_t(1) << nin)) return fail(p->ctx, OWQS_E_INVALID_ARG, "input size must be 2^(number of inputs)");
    if (nin > 0 && !input) return fail(p->ctx, OWQS_E_INVALID_ARG, "null input");
    const int32_t k = (int32_t)nin;
    return run_substates(p, &input, &k, nin ? 1 : 0, input_on_device, stream, prof);
  }
  if (p && p->sampling) {
    if (prof) return fail(p->ctx, OWQS_E_STATE, "profiled runs take forced outcomes");
    return run_sampled(p, input, n_amps, input_on_device, stream);
  }
  if (!p) return OWQS_E_INVALID_ARG;
  const size_t nin = p->inputs.size();
  if (owqs_status w = width_guard(p)) return w;
  const size_t want = size_t(1) << nin;
  if (n_amps != want) return fail(p->ctx, OWQS_E_INVALID_ARG, "input size must be 2^(number of inputs)");
  if (nin > 0 && !input) return fail(p->ctx, OWQS_E_INVALID_ARG, "null input");
  owqs_status st = ensure_device(p);
  if (st != OWQS_OK) return st;
  if (p->dirty) compile(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  end_ranged(p);
  p->sampled_ran = false;
  hipError_t e = launch_init(p->psi, p->book, s, nin == 0 && input == nullptr ? 1 : 0);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "init");
  if (nin > 0 || input != nullptr) {
    e = hipMemcpyAsync(p->psi, input, want * sizeof(float2),
                       input_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "input copy");
  }
  const int reduce = p->mode == OWQS_MODE_OWQS ? kReduceRenorm
                     : p->mode == OWQS_MODE_EOWQS_CHECK ? kReduceCheck
                                                        : kReduceNone;
  if (!prof && p->exec == OWQS_EXEC_AUTO && p->plan_width <= kLdsMaxWidth) {
    // whole pattern in one workgroup's LDS; the ordered, scaled read-out is
    // written to psi[0 .. 2^nout) (the input was read into LDS first)
    st = upload_steps(p);
    if (st != OWQS_OK) return st;
    // (the input, or the empty product state set by the init kernel, is in psi)
    LdsItem proto = lds_proto(p);
    proto.in = p->psi;
    proto.out = p->psi;
    proto.probs = p->book.probs;
    proto.err = p->book.err;
    e = launch_lds_shared(proto, 1, p->plan_width, reduce, 0, 0, (size_t)p->n_meas, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "LDS run");
    p->ran = true;
  p->ss_ran = false;
    p->out_in_order = true;
    p->batch_ran = false;
    p->ran_mode = reduce;
    return OWQS_OK;
  }
  p->out_in_order = false;
  st = upload_fuse(p);
  if (st != OWQS_OK) return st;
  // profiling: ev[2i] before step i's main kernel, ev[2i+1] after it (before
  // the FP64 finishing kernel, if any), ev[2i+2] after the step
  std::vector<hipEvent_t> ev;
  if (prof) {
    ev.resize(2 * p->xsteps.size() + 1);
    for (auto &x : ev) {
      e = hipEventCreate(&x);
      if (e != hipSuccess) return hip_fail(p->ctx, e, "event");
    }
    e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = launch_steps(p, reduce, s, &ev);
  } else if (p->use_graph && !p->xsteps.empty()) {
    if (!p->graph_exec) {
      if (!p->cap_stream) {
        e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "capture stream");
      }
      e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(p->ctx, e, "begin capture");
      hipError_t le = launch_steps(p, reduce, p->cap_stream, nullptr);
      e = hipStreamEndCapture(p->cap_stream, &p->graph);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
        p->graph_exec = nullptr;
        return hip_fail(p->ctx, e, "graph capture");
      }
      p->graph_reduce = reduce;
    }
    e = hipGraphLaunch(p->graph_exec, s);
  } else {
    e = launch_steps(p, reduce, s, nullptr);
  }
  if (e != hipSuccess) {
    for (auto &x : ev) (void)hipEventDestroy(x);
    return hip_fail(p->ctx, e, "kernel launch");
  }
  p->ran = true;
  p->ss_ran = false;
  p->batch_ran = false;
  p->ran_mode = reduce;
  if (prof) {
    e = hipStreamSynchronize(s);
    for (size_t i = 0; i < p->xsteps.size() && e == hipSuccess; ++i) {
      float t = 0.f, f = 0.f;
      e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&f, ev[2 * i + 1], ev[2 * i + 2]);
      const int k = p->xsteps[i].kind;
      prof->counts[k] += 1;
      prof->ms[k] += t;
      prof->bytes[k] += step_bytes(p->xsteps[i]);
      // a half group without renorm launches no finishing kernel
      const bool half = half_prob(p->xsteps[i], reduce) ||
                        (k == S_F && reduce == kReduceRenorm && p->groups[p->xsteps[i].group].half &&
                         !p->groups[p->xsteps[i].group].renorm);
      if ((k == S_M || k == S_J || k == S_F) && reduce != kReduceNone && !half) {
        prof->counts[OWQS_KIND_FINISH] += 1;
        prof->ms[OWQS_KIND_FINISH] += f;
      }
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "profile events");
  }
  return OWQS_OK;
}

// ---- text format v1 ----
bool parse_text(const char *text, size_t len, std::vector<owqs_cmd> &cmds, std::vector<int32_t> &dom,
                std::vector<int32_t> &ins, std::vector<int32_t> &outs, std::string &err) {
  std::string all(text, len);
  size_t pos = 0;
  int lineno = 0;
  while (pos <= all.size()) {
    size_t eol = all.find('\n', pos);
    if (eol == std::string::npos) eol = all.size();
    std::string line = all.substr(pos, eol - pos);
    pos = eol + 1;
    ++lineno;
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::vector<std::string> tok;
    {
      size_t a = 0;
      while (a < line.size()) {
        while (a < line.size() && isspace((unsigned char)line[a])) ++a;
        size_t b = a;
        while (b < line.size() && !isspace((unsigned char)line[b])) ++b;
        if (b > a) tok.push_back(line.substr(a, b - a));
        a = b;
      }
    }
    if (tok.empty()) {
      if (eol == all.size()) break;
      continue;
    }
    auto to_int = [&](const std::string &s, int32_t &v) {
      char *end = nullptr;
      const long x = strtol(s.c_str(), &end, 10);
      if (!end || *end || x < INT32_MIN || x > INT32_MAX) return false;
      v = (int32_t)x;
      return true;
    };
    const std::string &h = tok[0];
    auto bad = [&](const char *why) {
      err = "line " + std::to_string(lineno) + ": " + why;
      return false;
    };
    if (h == "inputs" || h == "outputs") {
      auto &dst = (h == "inputs") ? ins : outs;
      for (size_t k = 1; k < tok.size(); ++k) {
        int32_t v;
        if (!to_int(tok[k], v)) return bad("bad qubit id");
        dst.push_back(v);
      }
      continue;
    }
    owqs_cmd c{};
    int32_t v;
    if (h == "N") {
      if (tok.size() != 2 || !to_int(tok[1], v)) return bad("N takes one qubit");
      c.op = OWQS_OP_N;
      c.q0 = v;
    } else if (h == "E") {
      int32_t w;
      if (tok.size() != 3 || !to_int(tok[1], v) || !to_int(tok[2], w)) return bad("E takes two qubits");
      c.op = OWQS_OP_E;
      c.q0 = v;
      c.q1 = w;
    } else if (h == "M" || h == "X" || h == "Z") {
      if (tok.size() < 2 || !to_int(tok[1], v)) return bad("missing qubit");
      c.op = h == "M" ? OWQS_OP_M : (h == "X" ? OWQS_OP_X : OWQS_OP_Z);
      c.q0 = v;
      size_t k = 2;
      if (c.op == OWQS_OP_M) {
        if (tok.size() < 3) return bad("M needs an angle");
        char *end = nullptr;
        c.angle = strtod(tok[2].c_str(), &end);
        if (!end || *end) return bad("bad angle");
        k = 3;
      }
      int which = -1;  // 0 = s, 1 = t
      std::vector<int32_t> sd, td;
      for (; k < tok.size(); ++k) {
        if (tok[k] == "s:") { which = 0; continue; }
        if (tok[k] == "t:") {
          if (c.op != OWQS_OP_M) return bad("t-domain on a correction");
          which = 1;
          continue;
        }
        if (which < 0 || !to_int(tok[k], v)) return bad("bad domain");
        (which == 0 ? sd : td).push_back(v);
      }
      c.s_off = (int32_t)dom.size();
      c.s_len = (int32_t)sd.size();
      dom.insert(dom.end(), sd.begin(), sd.end());
      c.t_off = (int32_t)dom.size();
      c.t_len = (int32_t)td.size();
      dom.insert(dom.end(), td.begin(), td.end());
    } else {
      return bad("unknown command");
    }
    cmds.push_back(c);
    if (eol == all.size()) break;
  }
  return true;
}

}  // namespace owqs

// ===========================================================================
// C ABI
// ===========================================================================
namespace owqs {

void pattern_export(const owqs_pattern *p, std::vector<owqs_cmd> &cmds, std::vector<int32_t> &dom,
                    std::vector<int32_t> &inputs, std::vector<int32_t> &outputs) {
  cmds.clear();
  dom.clear();
  inputs.clear();
  outputs.clear();
  for (int q : p->inputs) inputs.push_back(p->user_id[q]);
  for (int q : p->outputs) outputs.push_back(p->user_id[q]);
  size_t m = 0;
  for (const Cmd &c : p->cmds) {
    owqs_cmd o{};
    o.op = c.op;
    o.q0 = p->user_id[c.q0];
    o.q1 = c.op == OWQS_OP_E ? p->user_id[c.q1] : 0;
    o.s_off = (int32_t)dom.size();
    for (int q : c.s) dom.push_back(p->user_id[q]);
    o.s_len = (int32_t)c.s.size();
    o.t_off = (int32_t)dom.size();
    for (int q : c.t) dom.push_back(p->user_id[q]);
    o.t_len = (int32_t)c.t.size();
    if (c.op == OWQS_OP_M) o.angle = p->angles[m++];
    cmds.push_back(o);
  }
}

owqs_ctx *pattern_ctx(const owqs_pattern *p) { return p->ctx; }

owqs_status pattern_fail(const owqs_pattern *p, owqs_status st, const std::string &msg) {
  return fail(p->ctx, st, msg);
}

}  // namespace owqs

extern "C" {

const char *owqs_status_str(owqs_status s) {
  switch (s) {
    case OWQS_OK: return "OWQS_OK";
    case OWQS_E_INVALID_ARG: return "OWQS_E_INVALID_ARG";
    case OWQS_E_PATTERN: return "OWQS_E_PATTERN";
    case OWQS_E_ZERO_PROB: return "OWQS_E_ZERO_PROB";
    case OWQS_E_WIDTH: return "OWQS_E_WIDTH";
    case OWQS_E_NOMEM: return "OWQS_E_NOMEM";
    case OWQS_E_HIP: return "OWQS_E_HIP";
    case OWQS_E_NOT_DETERMINISTIC: return "OWQS_E_NOT_DETERMINISTIC";
    case OWQS_E_STATE: return "OWQS_E_STATE";
  }
  return "OWQS_UNKNOWN";
}

owqs_status owqs_ctx_create(int device, owqs_ctx **out) {
  if (!out) return OWQS_E_INVALID_ARG;
  if (device != -1) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) return OWQS_E_INVALID_ARG;
  }
  void *scratch = nullptr;
  if (device >= 0) {
    // resolve the allocation-free entry point's array once per device, with
    // that device current (then restore the caller's current device)
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e == hipSuccess) e = noalloc_scratch(device, &scratch);
    if (e == hipSuccess) e = hipSetDevice(prev);
    if (e != hipSuccess) return OWQS_E_HIP;
  }
  auto *c = new owqs_ctx();
  c->device = device;
  c->noalloc = scratch;
  *out = c;
  return OWQS_OK;
}

void owqs_ctx_destroy(owqs_ctx *ctx) {
  if (!ctx) return;
  owqs_ctx::Batch &b = ctx->batch;
  if (ctx->device >= 0 && (b.exec || b.graph || b.dev || b.cap || b.done)) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    if (b.dev) (void)hipFree(b.dev);
    if (b.cap) (void)hipStreamDestroy(b.cap);
    for (int c = 0; c < 5; ++c) {
      if (b.side[c]) (void)hipStreamDestroy(b.side[c]);
      if (b.join[c]) (void)hipEventDestroy(b.join[c]);
    }
    if (b.fork) (void)hipEventDestroy(b.fork);
    if (b.done) (void)hipEventDestroy(b.done);
  }
  delete ctx;
}

const char *owqs_last_error(const owqs_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

owqs_status owqs_pattern_create(owqs_ctx *ctx, const owqs_cmd *cmds, size_t ncmds, const int32_t *domain_ids,
                                size_t ndom, const int32_t *inputs, int32_t nin, const int32_t *outputs,
                                int32_t nout, owqs_pattern **out) {
  if (cmds)
    for (size_t i = 0; i < ncmds; ++i)
      if (cmds[i].reserved != 0) return fail(ctx, OWQS_E_INVALID_ARG, "owqs_cmd.reserved must be 0");
  return build_pattern(ctx, cmds, ncmds, domain_ids, ndom, inputs, nin, outputs, nout, out);
}

owqs_status owqs_pattern_from_text(owqs_ctx *ctx, const char *text, size_t len, owqs_pattern **out) {
  if (!ctx || !text || !out) return fail(ctx, OWQS_E_INVALID_ARG, "null pointer");
  std::vector<owqs_cmd> cmds;
  std::vector<int32_t> dom, ins, outs;
  std::string err;
  if (!parse_text(text, len, cmds, dom, ins, outs, err)) return fail(ctx, OWQS_E_INVALID_ARG, err);
  return build_pattern(ctx, cmds.data(), cmds.size(), dom.data(), dom.size(), ins.data(), (int32_t)ins.size(),
                       outs.data(), (int32_t)outs.size(), out);
}

void owqs_pattern_destroy(owqs_pattern *p) {
  if (!p) return;
  if (p->psi || p->book_mem || p->stage || p->dev_steps || p->graph_exec || p->adj_mem || p->s_mem || p->ss_mem ||
      p->a_mem) {
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    if (p->psi) (void)hipFree(p->psi);
    if (p->book_mem) (void)hipFree(p->book_mem);
  }
  if (p->stage) (void)hipFree(p->stage);
  if (p->dev_steps) (void)hipFree(p->dev_steps);
  if (p->dev_fuse) (void)hipFree(p->dev_fuse);
  if (p->adj_mem) (void)hipFree(p->adj_mem);
  if (p->s_mem) (void)hipFree(p->s_mem);
  if (p->ss_mem) (void)hipFree(p->ss_mem);
  if (p->a_mem) (void)hipFree(p->a_mem);
  if (p->a_exec) (void)hipGraphExecDestroy(p->a_exec);
  if (p->a_graph) (void)hipGraphDestroy(p->a_graph);
  if (p->ss_sigma) (void)hipFree(p->ss_sigma);
  if (p->ss_dev_fuse) (void)hipFree(p->ss_dev_fuse);
  if (p->ss_stage) (void)hipFree(p->ss_stage);
  if (p->ss_exec) (void)hipGraphExecDestroy(p->ss_exec);
  if (p->ss_graph) (void)hipGraphDestroy(p->ss_graph);
  if (p->s_exec) (void)hipGraphExecDestroy(p->s_exec);
  if (p->s_graph) (void)hipGraphDestroy(p->s_graph);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

owqs_status owqs_pattern_info(const owqs_pattern *p, int32_t *n_meas, int32_t *max_live, int32_t *n_in,
                              int32_t *n_out, size_t *ncmds) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (n_meas) *n_meas = p->n_meas;
  if (max_live) *max_live = p->max_live;
  if (n_in) *n_in = (int32_t)p->inputs.size();
  if (n_out) *n_out = (int32_t)p->outputs.size();
  if (ncmds) *ncmds = p->cmds.size();
  return OWQS_OK;
}

owqs_status owqs_pattern_commands(const owqs_pattern *p, owqs_cmd *cmds, size_t cmd_cap, int32_t *domain_ids,
                                  size_t dom_cap, int32_t *inputs, int32_t *outputs, size_t *ncmds, size_t *ndom) {
  if (!p) return OWQS_E_INVALID_ARG;
  std::vector<owqs_cmd> c;
  std::vector<int32_t> d, in, out;
  pattern_export(p, c, d, in, out);
  if (ncmds) *ncmds = c.size();
  if (ndom) *ndom = d.size();
  if ((cmds && cmd_cap < c.size()) || (domain_ids && dom_cap < d.size()))
    return fail(p->ctx, OWQS_E_INVALID_ARG, "command or domain buffer too small");
  if (cmds && !c.empty()) std::memcpy(cmds, c.data(), c.size() * sizeof(owqs_cmd));
  if (domain_ids && !d.empty()) std::memcpy(domain_ids, d.data(), d.size() * sizeof(int32_t));
  if (inputs && !in.empty()) std::memcpy(inputs, in.data(), in.size() * sizeof(int32_t));
  if (outputs && !out.empty()) std::memcpy(outputs, out.data(), out.size() * sizeof(int32_t));
  return OWQS_OK;
}

owqs_status owqs_set_mode(owqs_pattern *p, owqs_mode mode) {
  if (!p || mode < OWQS_MODE_OWQS || mode > OWQS_MODE_EOWQS_CHECK) return OWQS_E_INVALID_ARG;
  if (p->mode != mode) p->dirty = true;
  p->mode = mode;
  return OWQS_OK;
}

owqs_status owqs_set_exec(owqs_pattern *p, owqs_exec exec) {
  if (!p || exec < OWQS_EXEC_PLAIN || exec > OWQS_EXEC_SUBSTATES) return OWQS_E_INVALID_ARG;
  if ((p->exec == OWQS_EXEC_PLAIN) != (exec == OWQS_EXEC_PLAIN)) p->dirty = true;
  if ((p->exec == OWQS_EXEC_SUBSTATES) != (exec == OWQS_EXEC_SUBSTATES)) p->dirty = true;
  p->exec = exec;
  return OWQS_OK;
}

owqs_status owqs_set_angles(owqs_pattern *p, const double *alpha, size_t n_meas) {
  if (!p || (n_meas && !alpha)) return OWQS_E_INVALID_ARG;
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "angle count != number of M commands");
  p->angles.assign(alpha, alpha + n_meas);
  p->dirty = true;
  p->s_valid = false;
  return OWQS_OK;
}

owqs_status owqs_set_outcomes(owqs_pattern *p, const uint8_t *bits, size_t n_meas) {
  if (!p || (n_meas && !bits)) return OWQS_E_INVALID_ARG;
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "outcome count != number of M commands");
  for (size_t k = 0; k < n_meas; ++k)
    if (bits[k] > 1) return fail(p->ctx, OWQS_E_INVALID_ARG, "outcomes must be 0 or 1");
  p->outcomes.assign(bits, bits + n_meas);
  p->dirty = true;
  p->sampling = false;
  return OWQS_OK;
}

owqs_status owqs_run(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device, void *stream) {
  return run_impl(p, input, n_amps, input_on_device, stream, nullptr);
}

owqs_status owqs_run_profiled(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device,
                              void *stream, int64_t *counts, double *ms, double *bytes) {
  if (!counts || !ms || !bytes) return OWQS_E_INVALID_ARG;
  Profile prof{counts, ms, bytes};
  return run_impl(p, input, n_amps, input_on_device, stream, &prof);
}

owqs_status owqs_set_graph(owqs_pattern *p, int enable) {
  if (!p) return OWQS_E_INVALID_ARG;
  p->use_graph = enable != 0;
  return OWQS_OK;
}

owqs_status owqs_set_sum_all(owqs_pattern *p, int32_t on) {
  if (!p || (on != 0 && on != 1)) return OWQS_E_INVALID_ARG;
  const int cap = on ? 0 : kHalfRun;
  if (p->half_cap != cap) {
    p->half_cap = cap;
    p->dirty = true;
    p->s_valid = false;  // the drawn-outcome plan decides its windows' sums too
  }
  return OWQS_OK;
}

owqs_status owqs_set_tile_bits(owqs_pattern *p, int32_t bits) {
  if (!p || (bits != 0 && (bits < 10 || bits > kMaxTileBits))) return OWQS_E_INVALID_ARG;
  if (p->tile_bits != bits) p->dirty = true;
  p->tile_bits = bits;
  return OWQS_OK;
}

owqs_status owqs_tune(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device, void *stream,
                      int32_t *best_bits, float *best_ms) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (substates(p)) return refuse_substates(p, "owqs_tune");
  if (owqs_status w = width_guard(p)) return w;
  if (p->dirty) compile(p);
  // only plans with tile passes have a schedule to choose
  bool tiled = p->exec != OWQS_EXEC_PLAIN && !(p->exec == OWQS_EXEC_AUTO && p->plan_width <= kLdsMaxWidth);
  if (tiled) {
    tiled = false;
    for (const Step &x : p->steps) tiled |= x.n >= kTileMinWidth && (x.kind == S_J || x.kind == S_E);
  }
  if (!tiled) {
    if (best_bits) *best_bits = p->tile_bits;
    if (best_ms) *best_ms = 0.f;
    return OWQS_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "tune events");
  const int keep = p->tile_bits;
  int best = keep;
  float best_t = 0.f;
  owqs_status st = OWQS_OK;
  for (int bits = 10; bits <= kMaxTileBits && st == OWQS_OK; ++bits) {
    owqs_set_tile_bits(p, bits);
    st = owqs_run(p, input, n_amps, input_on_device, stream);  // capture / warm-up
    if (st != OWQS_OK) break;
    e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && st == OWQS_OK && e == hipSuccess; ++r)
      st = owqs_run(p, input, n_amps, input_on_device, stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) break;
    if (best_t == 0.f || t < best_t) {
      best_t = t;
      best = bits;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != OWQS_OK) {
    owqs_set_tile_bits(p, keep);
    return st;
  }
  if (e != hipSuccess) {
    owqs_set_tile_bits(p, keep);
    return hip_fail(p->ctx, e, "tune");
  }
  owqs_set_tile_bits(p, best);
  if (best_bits) *best_bits = best;
  if (best_ms) *best_ms = best_t / 3.f;
  return OWQS_OK;
}

owqs_status owqs_tune_batch(owqs_ctx *ctx, owqs_pattern *const *pats, size_t npat, const void *const *inputs,
                            void *const *outputs, void *stream, int32_t *best_bits, float *best_ms) {
  if (!ctx || (npat && (!pats || !outputs))) return fail(ctx, OWQS_E_INVALID_ARG, "null argument");
  if (ctx->device < 0) return fail(ctx, OWQS_E_STATE, "host-only context");
  // the patterns whose plans have tile passes in a batch (plan width > 14)
  std::vector<owqs_pattern *> wide;
  std::vector<int> keep;
  for (size_t i = 0; i < npat; ++i) {
    owqs_pattern *p = pats[i];
    if (!p || p->ctx != ctx) return fail(ctx, OWQS_E_INVALID_ARG, "pattern " + std::to_string(i));
    if (substates(p)) return refuse_substates(p, "owqs_tune_batch");
    if (owqs_status w = width_guard(p)) return w;
    if (p->dirty) compile(p);
    if (p->plan_width > kLdsMaxWidth && p->exec != OWQS_EXEC_PLAIN) {
      wide.push_back(p);
      keep.push_back(p->tile_bits);
    }
  }
  if (wide.empty()) {
    if (best_bits) *best_bits = 0;
    if (best_ms) *best_ms = 0.f;
    return OWQS_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "tune events");
  int best = -1;
  float best_t = 0.f;
  owqs_status st = OWQS_OK;
  for (int bits = 10; bits <= kMaxTileBits && st == OWQS_OK && e == hipSuccess; ++bits) {
    for (owqs_pattern *p : wide) owqs_set_tile_bits(p, bits);
    st = owqs_run_batch(ctx, pats, npat, inputs, outputs, stream);  // compile, capture, warm up
    if (st != OWQS_OK) break;
    e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && st == OWQS_OK && e == hipSuccess; ++r)
      st = owqs_run_batch(ctx, pats, npat, inputs, outputs, stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && st == OWQS_OK && (best < 0 || t < best_t)) {
      best_t = t;
      best = bits;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != OWQS_OK || e != hipSuccess) {
    for (size_t k = 0; k < wide.size(); ++k) owqs_set_tile_bits(wide[k], keep[k]);
    return st != OWQS_OK ? st : hip_fail(ctx, e, "tune");
  }
  for (owqs_pattern *p : wide) owqs_set_tile_bits(p, best);
  if (best_bits) *best_bits = best;
  if (best_ms) *best_ms = best_t / 3.f;
  return OWQS_OK;
}

owqs_status owqs_plan_info(owqs_pattern *p, int32_t *plan_width, size_t *nsteps, size_t *npasses) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (owqs_status w = width_guard(p)) return w;
  if (p->dirty) compile(p);
  if (plan_width) *plan_width = p->plan_width;
  if (nsteps) *nsteps = substates(p) ? p->ss_steps.size() : p->steps.size();
  if (npasses) *npasses = substates(p) ? p->ss_run.size() : p->xsteps.size();
  return OWQS_OK;
}

owqs_status owqs_plan_tile_work(owqs_pattern *p, size_t *windows, size_t *maps, size_t *composed) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (owqs_status w = width_guard(p)) return w;
  if (p->dirty) compile(p);
  size_t nw = 0, nm = 0, nc = 0;
  const int reduce = reduce_of(p);
  const bool ss = substates(p);
  const std::vector<TileGroup> &groups = ss ? p->ss_groups : p->groups;
  const std::vector<FuseOp> &fops = ss ? p->ss_fuse_ops : p->fuse_ops, &mops = ss ? p->ss_fuse_mops : p->fuse_mops;
  for (const TileGroup &tg : groups) {
    size_t gw = 0, gm = 0;
    // the commands a forced run launches (launch_range, launch_substeps): composed where the pass sums no window
    const bool comp = tg.mnops > 0 && (reduce == kReduceNone || (reduce == kReduceRenorm && tg.half));
    const FuseOp *ops = comp ? mops.data() + tg.mop_off : fops.data() + tg.op_off;
    const int nops = comp ? tg.mnops : tg.ta.nops;
    for (int i = 0; i < nops; ++i) {
      gw += ops[i].kind == DK_J;
      gm += ops[i].kind == DK_U;
    }
    nw += gw;
    nm += gm;
    nc += size_t(tg.ta.nwin) - gw;
  }
  if (windows) *windows = nw;
  if (maps) *maps = nm;
  if (composed) *composed = nc;
  return OWQS_OK;
}

static owqs_status run_shared(owqs_pattern *p, const void *in, uint32_t first, uint32_t count, void *out,
                              double *probs, void *stream, int basis_mode) {
  // every item runs the pattern's one command table in its own workgroup
  if (!p || !out) return OWQS_E_INVALID_ARG;
  if (substates(p)) return refuse_substates(p, basis_mode ? "owqs_run_basis" : "owqs_run_states");
  if (count == 0) return OWQS_OK;
  if (p->ctx->device < 0) return fail(p->ctx, OWQS_E_STATE, "host-only context");
  if (basis_mode && (p->inputs.size() > 31 || uint64_t(first) + count > (uint64_t(1) << p->inputs.size())))
    return fail(p->ctx, OWQS_E_INVALID_ARG, "basis range outside 2^(number of inputs)");
  if (!basis_mode && !in && !p->inputs.empty()) return fail(p->ctx, OWQS_E_INVALID_ARG, "null inputs");
  owqs_status st = ensure_device(p, false);
  if (st != OWQS_OK) return st;
  if (p->dirty) compile(p);
  if (p->plan_width > kLdsMaxWidth)
    return fail(p->ctx, OWQS_E_WIDTH, "plan width " + std::to_string(p->plan_width) + " exceeds the LDS limit 14");
  st = upload_steps(p);
  if (st != OWQS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  end_ranged(p);
  hipError_t e = launch_init(p->psi, p->book, s, 0);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "init");
  LdsItem proto = lds_proto(p);
  proto.in = static_cast<const float2 *>(in);
  if (!basis_mode && !in) {
    // only reachable with nin = 0 (checked above): every item starts from the
    // empty product state
    basis_mode = 1;
    first = 0;
    if (count != 1) return fail(p->ctx, OWQS_E_INVALID_ARG, "without inputs a pattern has a single input state");
  }
  proto.out = static_cast<float2 *>(out);
  proto.probs = probs;
  const int reduce = reduce_of(p);
  proto.err = p->book.err;
  e = launch_lds_shared(proto, (int)count, p->plan_width, reduce, first, basis_mode, (size_t)p->n_meas, s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "LDS kernel");
  p->ran = false;  // the pattern's own state buffer was not written
  p->ss_ran = false;
  p->batch_ran = true;
  return OWQS_OK;
}

owqs_status owqs_run_basis(owqs_pattern *p, uint32_t first, uint32_t count, void *out_c64, double *probs,
                           void *stream) {
  return run_shared(p, nullptr, first, count, out_c64, probs, stream, 1);
}

owqs_status owqs_run_states(owqs_pattern *p, const void *in_c64, uint32_t count, void *out_c64, double *probs,
                            void *stream) {
  return run_shared(p, in_c64, 0, count, out_c64, probs, stream, 0);
}

// ---- batched runs
//
// A batch is captured once as a graph and replayed while the call's arguments
// and every pattern's plan stay the same.  Patterns whose plan fits one
// workgroup's LDS (plan width <= 14) run whole in k_lds_batch, one launch per
// width class sized for that class; the others run level by level: level s
// applies the s-th step of every wide plan, with the tile groups of all
// patterns at that level in one k_tile_multi launch per tile shape and their
// group finishes in one k_finish_multi launch (other steps, and groups too
// large for the per-tile partials, launch per pattern).  One launch starts
// every wide pattern (input, sigma, error word) and one reads every output.
// The LDS-resident launches run on a branch of the graph beside the levels.

namespace owqs {
namespace {

// Width classes of the LDS-resident items: their launches size LDS and
// threads for the widest item of the class.
int lds_class(int width) { return width <= 8 ? 0 : width <= 11 ? 1 : width - 10; }  // 0..4
constexpr int kLdsClasses = 5;
static_assert(sizeof(owqs_ctx::Batch::side) / sizeof(hipStream_t) == kLdsClasses, "one branch per class");

struct Region {
  size_t off = 0;
  size_t bytes = 0;
};

size_t place(size_t &top, size_t bytes) {
  const size_t off = (top + 255) & ~size_t(255);
  top = off + bytes;
  return off;
}

void drop_batch_graph(owqs_ctx *ctx) {
  owqs_ctx::Batch &b = ctx->batch;
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.key.clear();
  b.nodes = 0;
}

hipError_t batch_streams(owqs_ctx *ctx) {
  owqs_ctx::Batch &b = ctx->batch;
  hipError_t e = hipSuccess;
  if (!b.cap) e = hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking);
  for (int c = 0; c < kLdsClasses && e == hipSuccess; ++c) {
    if (!b.side[c]) e = hipStreamCreateWithFlags(&b.side[c], hipStreamNonBlocking);
    if (e == hipSuccess && !b.join[c]) e = hipEventCreateWithFlags(&b.join[c], hipEventDisableTiming);
  }
  if (e == hipSuccess && !b.fork) e = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming);
  if (e == hipSuccess && !b.done) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
  return e;
}

}  // namespace
}  // namespace owqs

owqs_status owqs_run_batch(owqs_ctx *ctx, owqs_pattern *const *pats, size_t npat, const void *const *inputs,
                           void *const *outputs, void *stream) {
  if (!ctx || (npat && (!pats || !outputs))) return fail(ctx, OWQS_E_INVALID_ARG, "null argument");
  for (size_t i = 0; i < npat; ++i)
    if (pats[i] && pats[i]->sampling)
      return fail(ctx, OWQS_E_STATE, "batched runs take forced outcomes (pattern " + std::to_string(i) + " draws them)");
  if (ctx->device < 0) return fail(ctx, OWQS_E_STATE, "host-only context");
  if (npat == 0) return OWQS_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    std::vector<const owqs_pattern *> seen(pats, pats + npat);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
      return fail(ctx, OWQS_E_INVALID_ARG, "a pattern appears twice in one batch");
  }
  // compile, place and upload every plan; the key of the call
  std::vector<size_t> lds, wide;
  std::vector<uint64_t> key;
  key.reserve(npat * 8);
  for (size_t i = 0; i < npat; ++i) {
    owqs_pattern *p = pats[i];
    if (!p || p->ctx != ctx || !outputs[i]) return fail(ctx, OWQS_E_INVALID_ARG, "pattern " + std::to_string(i));
    if (!p->inputs.empty() && (!inputs || !inputs[i])) return fail(ctx, OWQS_E_INVALID_ARG, "null input");
    if (substates(p)) return refuse_substates(p, "owqs_run_batch");
    if (owqs_status w = width_guard(p)) return w;
    if (p->dirty) compile(p);
    const bool in_lds = p->plan_width <= kLdsMaxWidth;
    owqs_status st = ensure_device(p, !in_lds);
    if (st == OWQS_OK) st = in_lds ? upload_steps(p) : upload_fuse(p);
    if (st != OWQS_OK) return st;
    (in_lds ? lds : wide).push_back(i);
    const uint64_t k[] = {uint64_t(uintptr_t(p)), p->plan_gen, uint64_t(uintptr_t(p->psi)),
                          uint64_t(uintptr_t(p->book_mem)), uint64_t(uintptr_t(in_lds ? (void *)p->dev_steps
                                                                                        : (void *)p->dev_fuse)),
                          uint64_t(uintptr_t(inputs ? inputs[i] : nullptr)), uint64_t(uintptr_t(outputs[i])),
                          uint64_t(reduce_of(p))};
    key.insert(key.end(), k, k + 8);
  }
  owqs_ctx::Batch &B = ctx->batch;
  if (!(B.exec && key == B.key)) {
    // ---- build: tables on the host, then one capture
    if (B.done) {
      e = hipEventSynchronize(B.done);  // a replay in flight still reads the old tables
      if (e != hipSuccess) return hip_fail(ctx, e, "previous batch");
    }
    drop_batch_graph(ctx);
    e = batch_streams(ctx);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch streams");
    static const hipError_t lds_prep = lds_batch_prepare();  // once per process, outside any capture
    if (lds_prep != hipSuccess) return hip_fail(ctx, lds_prep, "LDS batch kernel attribute");
    // LDS-resident items by width class, longest first within a class
    std::vector<LdsItem> cls_items[kLdsClasses];
    int cls_width[kLdsClasses] = {0, 0, 0, 0, 0};
    for (size_t i : lds) {
      owqs_pattern *p = pats[i];
      LdsItem it = lds_proto(p);
      it.in = inputs ? static_cast<const float2 *>(inputs[i]) : nullptr;
      if (p->inputs.empty() && !it.in) it.basis = 0;  // empty product state
      it.out = static_cast<float2 *>(outputs[i]);
      it.probs = p->book.probs;
      it.err = p->book.err;
      it.reduce = reduce_of(p);
      const int c = lds_class(p->plan_width);
      cls_items[c].push_back(it);
      cls_width[c] = std::max(cls_width[c], p->plan_width);
    }
    for (auto &v : cls_items)
      std::stable_sort(v.begin(), v.end(), [](const LdsItem &a, const LdsItem &b) {
        return ((size_t)a.nsteps << std::max(a.nin, a.nout)) > ((size_t)b.nsteps << std::max(b.nin, b.nout));
      });
    // start / read rows: wide patterns first (they are read out), then the
    // LDS-resident ones (only their error word is cleared)
    std::vector<BatchIo> ios;
    int max_nin = 0, max_nout = 0;
    for (size_t i : wide) {
      owqs_pattern *p = pats[i];
      BatchIo b{};
      b.psi = p->psi;
      b.in = inputs ? static_cast<const float2 *>(inputs[i]) : nullptr;
      b.out = static_cast<float2 *>(outputs[i]);
      b.book = p->book;
      b.final_factor = p->final_factor;
      b.nin = (int)p->inputs.size();
      b.nout = (int)p->outputs.size();
      b.reduce = reduce_of(p);
      for (size_t k = 0; k < p->final_where.size(); ++k) b.where[k] = p->final_where[k];
      max_nin = std::max(max_nin, b.nin);
      max_nout = std::max(max_nout, b.nout);
      ios.push_back(b);
    }
    for (size_t i : lds) {
      BatchIo b{};
      b.book = pats[i]->book;
      ios.push_back(b);
    }
    // levels of the wide plans
    struct Bucket {
      int k;
      bool runs, red, maps;
      std::vector<MultiTile> ents;
      uint32_t total = 0;
    };
    struct Level {
      std::vector<Bucket> buckets;
      std::vector<MultiFinish> fins;
      int maxwin = 0;
      std::vector<size_t> solo;  // wide patterns whose step runs on its own launches
    };
    size_t depth = 0;
    for (size_t i : wide) depth = std::max(depth, pats[i]->xsteps.size());
    std::vector<Level> levels(depth);
    for (size_t lv = 0; lv < depth; ++lv) {
      Level &L = levels[lv];
      for (size_t i : wide) {
        owqs_pattern *p = pats[i];
        if (lv >= p->xsteps.size()) continue;
        const Step &x = p->xsteps[lv];
        const int reduce = reduce_of(p);
        bool multi = false;
        if (x.kind == S_F) {
          const TileGroup &tg = p->groups[x.group];
          const uint64_t ntiles = uint64_t(1) << (tg.ta.n - tg.ta.k);
          const int r = (reduce == kReduceRenorm && tg.half) ? kReduceNone : reduce;
          multi = ntiles <= kTileGridCap && tg.ta.nwin <= (r != kReduceNone ? kMaxGroupWindows : kMaxHalfWindows);
          if (multi) {
            MultiTile m{};
            m.psi = p->psi;
            m.ops = p->dev_fuse + tg.op_off;
            m.partials = p->book.partials;
            m.sigma = p->book.sigma;
            m.probs = p->book.probs;
            m.ta = tg.ta;
            const bool renorm = r == kReduceNone && reduce == kReduceRenorm && tg.renorm;
            if (r == kReduceNone && reduce == kReduceRenorm) m.ta.half_m = fuse_m_dev(p) + tg.m_off;
            m.ta.renorm = renorm ? 1 : 0;
            m.reduce = r;
            if (tg.mnops > 0 && r == kReduceNone) {  // no window sums: the composed commands
              m.ops = p->dev_fuse + fuse_mops_base(p->fuse_ops.size(), p->fuse_m.size()) + tg.mop_off;
              m.ta.nops = tg.mnops;
              m.ta.maps = 1;
            }
            Bucket *bk = nullptr;
            const bool red = r != kReduceNone, maps = m.ta.maps != 0;
            for (Bucket &b : L.buckets)
              if (b.k == tg.ta.k && b.runs == (tg.ta.runs != 0) && b.red == red && b.maps == maps) bk = &b;
            if (!bk) {
              L.buckets.push_back(Bucket{tg.ta.k, tg.ta.runs != 0, red, maps, {}, 0});
              bk = &L.buckets.back();
            }
            m.first_tile = bk->total;
            bk->total += uint32_t(ntiles);
            bk->ents.push_back(m);
            if ((r != kReduceNone || renorm) && tg.ta.nwin > 0) {
              MultiFinish f{};
              f.book = p->book;
              f.m_of_window = fuse_m_dev(p) + tg.m_off;
              f.nwin = renorm ? 1 : tg.ta.nwin;
              f.reduce = r;
              f.ntiles = uint32_t(ntiles);
              f.renorm = renorm ? 1 : 0;
              L.fins.push_back(f);
              L.maxwin = std::max(L.maxwin, f.nwin);
            }
          }
        }
        if (!multi) L.solo.push_back(i);
      }
    }
    // one device image of every table
    size_t top = 0;
    size_t cls_off[kLdsClasses];
    for (int c = 0; c < kLdsClasses; ++c) cls_off[c] = place(top, cls_items[c].size() * sizeof(LdsItem));
    const size_t io_off = place(top, ios.size() * sizeof(BatchIo));
    std::vector<std::vector<size_t>> bk_off(depth);
    std::vector<size_t> fin_off(depth);
    for (size_t lv = 0; lv < depth; ++lv) {
      for (Bucket &b : levels[lv].buckets) bk_off[lv].push_back(place(top, b.ents.size() * sizeof(MultiTile)));
      fin_off[lv] = place(top, levels[lv].fins.size() * sizeof(MultiFinish));
    }
    std::vector<char> image(std::max<size_t>(top, 1), 0);
    for (int c = 0; c < kLdsClasses; ++c)
      if (!cls_items[c].empty())
        std::memcpy(image.data() + cls_off[c], cls_items[c].data(), cls_items[c].size() * sizeof(LdsItem));
    if (!ios.empty()) std::memcpy(image.data() + io_off, ios.data(), ios.size() * sizeof(BatchIo));
    for (size_t lv = 0; lv < depth; ++lv) {
      for (size_t q = 0; q < levels[lv].buckets.size(); ++q) {
        const Bucket &b = levels[lv].buckets[q];
        std::memcpy(image.data() + bk_off[lv][q], b.ents.data(), b.ents.size() * sizeof(MultiTile));
      }
      if (!levels[lv].fins.empty())
        std::memcpy(image.data() + fin_off[lv], levels[lv].fins.data(), levels[lv].fins.size() * sizeof(MultiFinish));
    }
    if (B.dev_cap < image.size()) {
      if (B.dev) (void)hipFree(B.dev);
      B.dev = nullptr;
      B.dev_cap = 0;
      e = hipMalloc(&B.dev, image.size());
      if (e != hipSuccess) return fail(ctx, OWQS_E_NOMEM, "batch tables");
      B.dev_cap = image.size();
    }
    e = hipMemcpy(B.dev, image.data(), image.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch table upload");
    char *dev = static_cast<char *>(B.dev);
    // ---- capture
    e = hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
    size_t nodes = 0;
    const BatchIo *dios = reinterpret_cast<const BatchIo *>(dev + io_off);
    hipError_t le = launch_batch_start(dios, (int)wide.size(), max_nin, B.cap);
    if (le == hipSuccess) le = launch_batch_start(dios + wide.size(), (int)lds.size(), 0, B.cap);
    nodes += (wide.empty() ? 0 : 1) + (lds.empty() ? 0 : 1);
    if (!lds.empty() && le == hipSuccess) le = hipEventRecord(B.fork, B.cap);
    bool forked[kLdsClasses] = {};
    for (int c = 0; c < kLdsClasses && le == hipSuccess; ++c) {  // each class a branch of its own
      if (cls_items[c].empty()) continue;
      le = hipStreamWaitEvent(B.side[c], B.fork, 0);
      forked[c] = le == hipSuccess;
      if (le == hipSuccess)
        le = launch_lds_batch(reinterpret_cast<const LdsItem *>(dev + cls_off[c]), (int)cls_items[c].size(),
                              cls_width[c], B.side[c]);
      if (le == hipSuccess) le = hipEventRecord(B.join[c], B.side[c]);
      ++nodes;
    }
    for (size_t lv = 0; lv < depth && le == hipSuccess; ++lv) {
      const Level &L = levels[lv];
      for (size_t q = 0; q < L.buckets.size() && le == hipSuccess; ++q) {
        const Bucket &b = L.buckets[q];
        le = launch_tile_multi(reinterpret_cast<const MultiTile *>(dev + bk_off[lv][q]), (int)b.ents.size(), b.total,
                               b.k, b.runs, b.red, b.maps, B.cap);
        ++nodes;
      }
      if (le == hipSuccess && !L.fins.empty()) {
        le = launch_finish_multi(reinterpret_cast<const MultiFinish *>(dev + fin_off[lv]), (int)L.fins.size(),
                                 L.maxwin, B.cap);
        ++nodes;
      }
      for (size_t j = 0; j < L.solo.size() && le == hipSuccess; ++j) {
        owqs_pattern *p = pats[L.solo[j]];
        le = launch_range(p, p->xsteps, lv, lv + 1, reduce_of(p), B.cap, nullptr);
        nodes += 2;
      }
    }
    if (le == hipSuccess) le = launch_batch_read(dios, (int)wide.size(), max_nout, B.cap);
    for (int c = 0; c < kLdsClasses && le == hipSuccess; ++c)
      if (!cls_items[c].empty()) le = hipStreamWaitEvent(B.cap, B.join[c], 0);
    if (le != hipSuccess)  // join every forked branch, so that the capture ends whole (the graph is dropped)
      for (int c = 0; c < kLdsClasses; ++c)
        if (forked[c] && hipEventRecord(B.join[c], B.side[c]) == hipSuccess)
          (void)hipStreamWaitEvent(B.cap, B.join[c], 0);
    nodes += wide.empty() ? 0 : 1;
    e = hipStreamEndCapture(B.cap, &B.graph);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_batch_graph(ctx);
      return hip_fail(ctx, e, "batch capture");
    }
    B.key = key;
    B.nodes = nodes;
  }
  e = hipGraphLaunch(B.exec, s);
  if (e == hipSuccess) e = hipEventRecord(B.done, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
  for (size_t i : lds) {
    owqs_pattern *p = pats[i];
    end_ranged(p);
    p->ran = false;
    p->ss_ran = false;
    p->sampled_ran = false;
    p->batch_ran = true;  // outputs went straight to the caller
  }
  for (size_t i : wide) {
    owqs_pattern *p = pats[i];
    end_ranged(p);
    p->ran = true;  // the live vector holds the result: owqs_read_state reads it again
    p->ss_ran = false;
    p->sampled_ran = false;
    p->batch_ran = false;
    p->out_in_order = false;
    p->ran_mode = reduce_of(p);
  }
  return OWQS_OK;
}

owqs_status owqs_check(owqs_pattern *p, void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (!p->ran && !p->batch_ran && !p->lk_ran) return fail(p->ctx, OWQS_E_STATE, "no run yet");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int err[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(err, p->book.err, sizeof(err), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "check");
  if (err[0] != kErrNone) {
    const bool zp = err[1] == kErrZeroProb;
    return fail(p->ctx, zp ? OWQS_E_ZERO_PROB : OWQS_E_NOT_DETERMINISTIC,
                std::string(zp ? "forced outcome with probability < 1e-10" : "|p - 1/2| > 1e-4") +
                    " at measurement (or batch item) " + std::to_string(err[0]));
  }
  return OWQS_OK;
}

owqs_status owqs_read_state(owqs_pattern *p, void *out, size_t n_amps, int out_on_device, void *stream) {
  if (!p || !out) return OWQS_E_INVALID_ARG;
  if (!p->ran)
    return fail(p->ctx, OWQS_E_STATE, p->lk_ran ? "the last run was a ranged run: read it with owqs_read_live"
                                                : "no run yet");
  const size_t nout = p->outputs.size();
  if (nout > OWQS_MAX_WIDTH)
    return fail(p->ctx, OWQS_E_WIDTH, "more outputs than OWQS_MAX_WIDTH: read the factors (owqs_read_substates)");
  if (n_amps != (size_t(1) << nout)) return fail(p->ctx, OWQS_E_INVALID_ARG, "output size must be 2^(outputs)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->ss_ran) {
    // the tensor product of the factors and the scalar, in output bit order
    std::vector<uint64_t> offs;
    owqs_status st = stage_substates(p, s, offs);
    if (st != OWQS_OK) return st;
    AssembleArgs aa{};
    aa.nf = (int)p->ss_factors.size();
    for (int f = 0; f < aa.nf; ++f) {
      aa.off[f] = offs[f];
      aa.mask[f] = p->ss_factors[f].mask;
    }
    aa.scalar_off = offs.back();
    hipError_t e = hipSuccess;
    float2 *dst = static_cast<float2 *>(out);
    if (!out_on_device) {
      if (!p->stage) {
        e = hipMalloc(reinterpret_cast<void **>(&p->stage), n_amps * sizeof(float2));
        if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "read staging buffer");
      }
      dst = p->stage;
    }
    e = launch_assemble(dst, (int)nout, p->ss_stage, aa, s);
    if (e == hipSuccess && !out_on_device) {
      e = hipMemcpyAsync(out, p->stage, n_amps * sizeof(float2), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return hip_fail(p->ctx, e, "read");
    return out_on_device ? OWQS_OK : owqs_check(p, stream);
  }
  const double *sigma = p->ran_mode == kReduceRenorm ? p->book.sigma : nullptr;
  const bool s_plan = p->sampled_ran && !p->an_ran;  // the drawn-window fused plan reads like a forced run
  const int *where = s_plan ? p->s_final_where.data() : p->final_where.data();
  const double factor = s_plan ? p->s_final_factor : p->final_factor;
  hipError_t e;
  if (p->out_in_order) {
    e = hipMemcpyAsync(out, p->psi, n_amps * sizeof(float2),
                       out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "read");
    if (out_on_device) return OWQS_OK;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "read");
    return owqs_check(p, stream);
  }
  if (out_on_device) {
    e = launch_read(p->psi, static_cast<float2 *>(out), (int)nout, where, factor, sigma, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "read");
    return OWQS_OK;
  }
  if (!p->stage) {
    e = hipMalloc(reinterpret_cast<void **>(&p->stage), n_amps * sizeof(float2));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "read staging buffer");
  }
  e = launch_read(p->psi, p->stage, (int)nout, where, factor, sigma, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, p->stage, n_amps * sizeof(float2), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "read");
  return owqs_check(p, stream);
}

owqs_status owqs_read_probs(owqs_pattern *p, double *probs, size_t n_meas, void *stream) {
  if (!p || (n_meas && !probs)) return OWQS_E_INVALID_ARG;
  if (!p->ran && !p->batch_ran && !p->lk_ran) return fail(p->ctx, OWQS_E_STATE, "no run yet");
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "probability count != M count");
  if (reduce_of(p) == kReduceNone) {
    for (size_t k = 0; k < n_meas; ++k) probs[k] = 0.5;
    return OWQS_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (n_meas) e = hipMemcpyAsync(probs, p->book.probs, n_meas * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "read probs");
  return OWQS_OK;
}

owqs_status owqs_run_range(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device,
                           size_t cmd_begin, size_t cmd_end, void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  const size_t nc = p->cmds.size();
  if (cmd_begin > cmd_end || cmd_end > nc) return fail(p->ctx, OWQS_E_INVALID_ARG, "command range outside the pattern");
  if (substates(p)) return refuse_substates(p, "owqs_run_range");
  owqs_status st = ensure_device(p);
  if (st != OWQS_OK) return st;
  if (p->dirty) compile(p);
  if (!p->lk_valid) {
    double ff = 1.0;
    std::vector<int> fw;
    PlanTrace tr{p->lk_step_end, p->lk_width, p->lk_pending, p->lk_qubits};
    compile_plan(p, false, p->lk_steps, fw, ff, &tr);
    p->lk_valid = true;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (cmd_begin == 0) {
    const size_t nin = p->inputs.size();
    const size_t want = size_t(1) << nin;
    if (n_amps != want) return fail(p->ctx, OWQS_E_INVALID_ARG, "input size must be 2^(number of inputs)");
    if (nin > 0 && !input) return fail(p->ctx, OWQS_E_INVALID_ARG, "null input");
    end_ranged(p);
    p->ran = false;
  p->ss_ran = false;
    p->batch_ran = false;
    p->out_in_order = false;
    e = launch_init(p->psi, p->book, s, nin == 0 && input == nullptr ? 1 : 0);
    if (e == hipSuccess && (nin > 0 || input != nullptr))
      e = hipMemcpyAsync(p->psi, input, want * sizeof(float2),
                         input_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "input");
  } else if (p->lk_next != cmd_begin) {
    return fail(p->ctx, OWQS_E_STATE, "a ranged run must start at 0 or where the previous ranged run ended");
  }
  const size_t i0 = cmd_begin ? p->lk_step_end[cmd_begin - 1] : 0;
  const size_t i1 = cmd_end ? p->lk_step_end[cmd_end - 1] : 0;
  p->lk_next = SIZE_MAX;  // set again only once the range is enqueued
  e = launch_range(p, p->lk_steps, i0, i1, reduce_of(p), s, nullptr);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "kernel launch");
  p->lk_next = cmd_end;
  p->lk_ran = true;
  p->ran_mode = reduce_of(p);
  return OWQS_OK;
}

owqs_status owqs_read_live(owqs_pattern *p, void *out_c64, size_t n_amps, int32_t *qubits, int32_t *n_live,
                           void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (!p->lk_ran || p->lk_next == SIZE_MAX) return fail(p->ctx, OWQS_E_STATE, "no ranged run to read");
  const size_t e_cmd = p->lk_next;
  const int n = e_cmd ? p->lk_width[e_cmd - 1] : (int)p->inputs.size();
  if (n_live) *n_live = n;
  if (qubits)
    for (int b = 0; b < n; ++b)
      qubits[b] = p->user_id[e_cmd ? p->lk_qubits[(e_cmd - 1) * kTraceStride + b] : p->inputs[b]];
  if (!out_c64) return OWQS_OK;
  if (n_amps != (size_t(1) << n)) return fail(p->ctx, OWQS_E_INVALID_ARG, "output size must be 2^(live width)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int where[OWQS_MAX_WIDTH + 1];
  for (int b = 0; b < n; ++b) where[b] = b;
  const double factor = e_cmd ? p->lk_pending[e_cmd - 1] : 1.0;
  const double *sigma = p->ran_mode == kReduceRenorm ? p->book.sigma : nullptr;
  float2 *tmp = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&tmp), n_amps * sizeof(float2));
  if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "live read buffer");
  e = launch_read(p->psi, tmp, n, where, factor, sigma, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out_c64, tmp, n_amps * sizeof(float2), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "live read");
  return owqs_check(p, stream);
}

}  // extern "C"

