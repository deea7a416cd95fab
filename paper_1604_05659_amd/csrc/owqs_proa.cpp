// owqs_proa.cpp -- pattern reordering (PROA, Sec. 4.3, Eq. 18) on the host.
//
// Input: a pattern whose corrections all follow its last measurement (the
// standard form, or any order that commutes to it).  Its E commands form the
// entanglement graph (an edge per odd number of E's).  By the Proposition of
// Sec. 4.3 a qubit only needs its own E's applied before it is measured, so
// the measurements can be chosen one at a time: every qubit starts in a
// singleton sub-state; measuring v merges the sub-states of v and of the
// neighbours it is not yet entangled with into its measurement state-space
// MS(v), after which v leaves that sub-state.  Among the ready qubits (every
// qubit of its signal domains already measured) the one of least cost is
// taken:
//   v touched before:  alpha |MS(v)| + beta OS(v) - gamma SS(v)
//   otherwise:         alpha (|MS(v)| + 1) delta + beta OS(v) - gamma SS(v)
// with OS(v) its edges to outputs and SS(v) the unmeasured qubits whose
// measurement depends on v; ties go to the smallest qubit id.  The default
// weights are |O|, |O|, 1/2, |O| with alpha swept from |O| down to 1 (Sec. 5),
// keeping the order whose largest state-space is smallest.
#include <algorithm>
#include <set>
#include <string>
#include <vector>

#include "owqs_pattern_access.h"

namespace owqs {
namespace {

struct Graph {
  int nq = 0;
  std::vector<int32_t> id;                 // dense -> caller's id
  std::vector<std::vector<int>> nbr;       // sorted by caller's id
  std::vector<std::vector<int>> deps;      // M domains (s and t), dense
  std::vector<char> is_out, is_in;
  std::vector<int> meas;                   // dense qubits measured, ascending caller id
  std::vector<int> m_cmd;                  // dense qubit -> index of its M command (-1)
};

struct Sweep {
  std::vector<int> order;
  int m = 0;
};

// One pass with fixed weights.  The ready qubits sit in a set ordered by
// (cost, id), so the first entry is the least cost with ties to the smallest
// id.  Measuring v changes only the costs of the qubits of its merged
// state-space, of their not-yet-entangled neighbours (whose MS holds that
// state-space) and of the qubits v depended on (their SS drops); those are
// re-keyed, and qubits whose last domain qubit was v join the set.
Sweep order_once(const Graph &g, double alpha, double beta, double gamma, double delta, bool free_order) {
  const int nq = g.nq;
  std::vector<int> sub(nq);                       // qubit -> sub-state id
  std::vector<std::vector<int>> members(nq);
  for (int q = 0; q < nq; ++q) {
    sub[q] = q;
    members[q] = {q};
  }
  std::vector<std::vector<int>> pending = g.nbr;  // neighbours not yet entangled
  std::vector<char> touched(nq, 0);
  std::vector<int> dependents(nq, 0);             // SS: unmeasured qubits whose domains hold q
  std::vector<int> waiting(nq, 0);                // unmeasured qubits in q's domains
  std::vector<std::vector<int>> needs_me(nq);     // q -> measured qubits whose domains hold q
  std::vector<int> os(nq, 0);                     // OS: edges to outputs
  for (int v : g.meas) {
    for (int d : g.deps[v]) {
      ++dependents[d];
      ++waiting[v];
      needs_me[d].push_back(v);
    }
    for (int u : g.nbr[v]) os[v] += g.is_out[u] ? 1 : 0;
  }
  std::vector<int> ids;
  auto ms_of = [&](int v) {
    ids.assign(1, sub[v]);
    for (int u : pending[v]) ids.push_back(sub[u]);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    int ms = 0;
    for (int s : ids) ms += (int)members[s].size();
    return ms;
  };
  auto cost_of = [&](int v) {
    const int ms = ms_of(v);
    return touched[v] ? alpha * ms + beta * os[v] - gamma * dependents[v]
                      : alpha * ((ms + 1) * delta) + beta * os[v] - gamma * dependents[v];
  };
  std::set<std::pair<double, int>> ready;
  std::vector<double> key(nq, 0.0);
  std::vector<char> queued(nq, 0);
  auto enqueue = [&](int v) {
    key[v] = cost_of(v);
    ready.insert({key[v], v});
    queued[v] = 1;
  };
  for (int v : g.meas)
    if (free_order || waiting[v] == 0) enqueue(v);
  std::vector<int> stamp(nq, -1), affected;
  Sweep out;
  for (size_t step = 0; step < g.meas.size(); ++step) {
    if (ready.empty()) return Sweep{};  // circular dependencies (validated patterns cannot have them)
    const int v = ready.begin()->second;
    ready.erase(ready.begin());
    queued[v] = 0;
    out.m = std::max(out.m, ms_of(v));
    out.order.push_back(v);
    // merge into v's state-space (ids holds its sub-states), then drop v
    std::vector<int> merged;
    for (int s : ids) {
      merged.insert(merged.end(), members[s].begin(), members[s].end());
      members[s].clear();
    }
    for (int q : merged) touched[q] = 1;
    merged.erase(std::remove(merged.begin(), merged.end(), v), merged.end());
    const int keep = ids[0];
    for (int q : merged) sub[q] = keep;
    members[keep] = merged;
    for (int u : pending[v]) {
      auto &pu = pending[u];
      pu.erase(std::remove(pu.begin(), pu.end(), v), pu.end());
    }
    pending[v].clear();
    for (int d : g.deps[v]) --dependents[d];
    // re-key what changed
    affected.clear();
    auto mark = [&](int q) {
      if (stamp[q] != (int)step) {
        stamp[q] = (int)step;
        affected.push_back(q);
      }
    };
    for (int q : merged) {
      mark(q);
      for (int u : pending[q]) mark(u);
    }
    for (int d : g.deps[v]) mark(d);
    for (int q : affected)
      if (queued[q]) {
        ready.erase({key[q], q});
        key[q] = cost_of(q);
        ready.insert({key[q], q});
      }
    if (!free_order)
      for (int u : needs_me[v])
        if (--waiting[u] == 0) enqueue(u);
  }
  return out;
}

}  // namespace
}  // namespace owqs

using namespace owqs;

extern "C" {

owqs_status owqs_pattern_reorder(const owqs_pattern *pat, const owqs_proa_opts *opts, owqs_pattern **out,
                                 owqs_proa_stats *stats) {
  if (!pat || !out) return OWQS_E_INVALID_ARG;
  if (opts && opts->reserved != 0) return pattern_fail(pat, OWQS_E_INVALID_ARG, "owqs_proa_opts.reserved must be 0");
  if (opts && opts->alpha > 0.0 && !(opts->beta >= 0.0 && opts->gamma >= 0.0 && opts->delta >= 0.0))
    return pattern_fail(pat, OWQS_E_INVALID_ARG, "reorder: weights must be non-negative");
  std::vector<owqs_cmd> cmds;
  std::vector<int32_t> dom;
  std::vector<int32_t> ins, outs;
  pattern_export(pat, cmds, dom, ins, outs);
  // every correction must follow every M and E: then the N's and E's commute
  // to the front and the M's may be taken in any order their domains allow
  bool seen_corr = false;
  for (const owqs_cmd &c : cmds) {
    if (c.op == OWQS_OP_X || c.op == OWQS_OP_Z) seen_corr = true;
    else if (seen_corr && (c.op == OWQS_OP_M || c.op == OWQS_OP_E))
      return pattern_fail(pat, OWQS_E_PATTERN,
                          "reorder: a correction comes before an M or E (pattern not in standard form)");
  }
  // dense graph over the caller's ids, ascending
  Graph g;
  std::vector<int32_t> all(ins);
  all.insert(all.end(), outs.begin(), outs.end());
  for (const owqs_cmd &c : cmds) {
    all.push_back(c.q0);
    if (c.op == OWQS_OP_E) all.push_back(c.q1);
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  g.nq = (int)all.size();
  g.id = all;
  auto dense = [&](int32_t q) { return int(std::lower_bound(all.begin(), all.end(), q) - all.begin()); };
  g.nbr.assign(g.nq, {});
  g.deps.assign(g.nq, {});
  g.is_out.assign(g.nq, 0);
  g.is_in.assign(g.nq, 0);
  g.m_cmd.assign(g.nq, -1);
  for (int32_t q : outs) g.is_out[dense(q)] = 1;
  for (int32_t q : ins) g.is_in[dense(q)] = 1;
  std::vector<std::vector<int>> count(g.nq);
  for (size_t i = 0; i < cmds.size(); ++i) {
    const owqs_cmd &c = cmds[i];
    if (c.op == OWQS_OP_E) {
      const int a = dense(c.q0), b = dense(c.q1);
      auto toggle = [&](int x, int y) {
        auto it = std::find(g.nbr[x].begin(), g.nbr[x].end(), y);
        if (it == g.nbr[x].end()) g.nbr[x].push_back(y);
        else g.nbr[x].erase(it);
      };
      toggle(a, b);
      toggle(b, a);
    } else if (c.op == OWQS_OP_M) {
      const int v = dense(c.q0);
      g.m_cmd[v] = (int)i;
      for (int32_t k = 0; k < c.s_len; ++k) g.deps[v].push_back(dense(dom[c.s_off + k]));
      for (int32_t k = 0; k < c.t_len; ++k) g.deps[v].push_back(dense(dom[c.t_off + k]));
    }
  }
  for (auto &n : g.nbr) std::sort(n.begin(), n.end());  // dense order = caller's id order
  for (auto &d : g.deps) {  // a domain is a set: a qubit listed twice (or in s and t) counts once
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
  }
  for (int q = 0; q < g.nq; ++q)
    if (g.m_cmd[q] >= 0) g.meas.push_back(q);
  const bool free_order = opts && opts->ignore_dependencies;
  Sweep best;
  double alpha_used = 0.0;
  const double no = std::max<double>((double)outs.size(), 1.0);
  if (opts && opts->alpha > 0.0) {
    best = order_once(g, opts->alpha, opts->beta, opts->gamma, opts->delta, free_order);
    alpha_used = opts->alpha;
  } else {
    bool have = false;
    for (int k = 0; k < (int)no; ++k) {
      const double a = no - k;
      Sweep s = order_once(g, a, no, 0.5, no, free_order);
      if (s.order.size() != g.meas.size()) continue;
      if (!have || s.m < best.m) {
        best = s;
        alpha_used = a;
        have = true;
      }
    }
  }
  if (best.order.size() != g.meas.size())
    return pattern_fail(pat, OWQS_E_PATTERN, "reorder: circular measurement dependencies");
  // the executable pattern: before measuring v, prepare v and the neighbours
  // it is not yet entangled with and apply those E's, then M v; afterwards
  // prepare the remaining outputs, apply the remaining E's, then the
  // corrections (dropped, with every domain, on the positive branch)
  std::vector<owqs_cmd> rc;
  std::vector<int32_t> rdom;
  std::vector<char> prepared(g.nq, 0);
  for (int q = 0; q < g.nq; ++q) prepared[q] = g.is_in[q];
  std::vector<std::vector<int>> pending = g.nbr;
  auto prep = [&](int q) {
    if (prepared[q]) return;
    owqs_cmd c{};
    c.op = OWQS_OP_N;
    c.q0 = g.id[q];
    rc.push_back(c);
    prepared[q] = 1;
  };
  auto copy_dom = [&](const owqs_cmd &src, owqs_cmd &dst) {
    dst.s_off = (int32_t)rdom.size();
    for (int32_t k = 0; k < src.s_len; ++k) rdom.push_back(dom[src.s_off + k]);
    dst.t_off = (int32_t)rdom.size();
    for (int32_t k = 0; k < src.t_len; ++k) rdom.push_back(dom[src.t_off + k]);
  };
  for (int v : best.order) {
    prep(v);
    for (int u : pending[v]) {
      prep(u);
      owqs_cmd e{};
      e.op = OWQS_OP_E;
      e.q0 = g.id[v];
      e.q1 = g.id[u];
      rc.push_back(e);
      auto &pu = pending[u];
      pu.erase(std::remove(pu.begin(), pu.end(), v), pu.end());
    }
    pending[v].clear();
    owqs_cmd m = cmds[g.m_cmd[v]];
    if (free_order) {
      m.s_off = m.s_len = m.t_off = m.t_len = 0;
    } else {
      copy_dom(cmds[g.m_cmd[v]], m);
    }
    rc.push_back(m);
  }
  for (int q = 0; q < g.nq; ++q)
    if (g.is_out[q]) prep(q);
  for (int q = 0; q < g.nq; ++q)
    for (int u : pending[q])
      if (u > q) {
        owqs_cmd e{};
        e.op = OWQS_OP_E;
        e.q0 = g.id[q];
        e.q1 = g.id[u];
        rc.push_back(e);
      }
  if (!free_order)
    for (const owqs_cmd &c : cmds)
      if (c.op == OWQS_OP_X || c.op == OWQS_OP_Z) {
        owqs_cmd x = c;
        copy_dom(c, x);
        x.t_off = x.t_len = 0;
        rc.push_back(x);
      }
  owqs_status st = owqs_pattern_create(pattern_ctx(pat), rc.data(), rc.size(), rdom.empty() ? nullptr : rdom.data(), rdom.size(),
                           ins.empty() ? nullptr : ins.data(), (int32_t)ins.size(),
                           outs.empty() ? nullptr : outs.data(), (int32_t)outs.size(), out);
  if (st != OWQS_OK) return st;
  if (stats) {
    stats->max_state_space = best.m;
    int32_t live = 0;
    owqs_pattern_info(*out, nullptr, &live, nullptr, nullptr, nullptr);
    stats->max_live = live;
    stats->alpha = alpha_used;
  }
  return OWQS_OK;
}

}  // extern "C"
