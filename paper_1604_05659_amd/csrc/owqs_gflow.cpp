// owqs_gflow.cpp -- EOWQS certificates and generalised flow (Sec. 4.5).
//
// EOWQS skips the probability of every measurement, which is exact when each
// outcome has probability 1/2.  For measurements in the XY plane that holds
// for measurement i whenever some set K of non-input qubits, all measured
// after i or outputs, has an odd neighbourhood that meets {i} and the qubits
// measured before i in exactly {i}: the graph-state stabiliser X_K Z_Odd(K)
// then commutes with every earlier measurement and anticommutes with i's, so
// i's outcome is an unbiased coin whatever the angles, the input and the
// earlier outcomes.  Such K are the sets g(i) of a generalised flow (gflow,
// reference [13] of the paper) whose order is the pattern's own.
//
// Finding K is a linear system over GF(2): unknown x_k for each candidate k,
// one equation per guarded qubit r (sum over k of adj(r, k) x_k = [r == i]).
// Only candidates adjacent to a guarded qubit and guarded qubits adjacent to a
// candidate enter it, so the systems stay the size of the frontier between
// measured and unmeasured qubits.
//
// owqs_pattern_gflow searches an order as well: starting from the outputs it
// adds, layer by layer, every qubit that the qubits already added (minus the
// inputs) can correct with the rest still unadded; a gflow exists when every
// qubit is added.  This is the layered construction of the maximally delayed
// gflow (the paper's reference [25]); a qubit's layer is the number of the
// round that added it (outputs: 0), and measuring higher layers first is an
// order with a witness for every qubit.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "owqs_pattern_access.h"

namespace owqs {
namespace {

struct OpenGraph {
  int nq = 0;
  std::vector<std::vector<int>> nbr;  // dense, sorted
  std::vector<char> is_in, is_out;
  std::vector<int> order;             // measured qubits, execution order
};

OpenGraph graph_of(const owqs_pattern *pat) {
  std::vector<owqs_cmd> cmds;
  std::vector<int32_t> dom, ins, outs;
  pattern_export(pat, cmds, dom, ins, outs);
  std::vector<int32_t> all(ins);
  all.insert(all.end(), outs.begin(), outs.end());
  for (const owqs_cmd &c : cmds) {
    all.push_back(c.q0);
    if (c.op == OWQS_OP_E) all.push_back(c.q1);
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  auto dense = [&](int32_t q) { return int(std::lower_bound(all.begin(), all.end(), q) - all.begin()); };
  OpenGraph g;
  g.nq = (int)all.size();
  g.nbr.assign(g.nq, {});
  g.is_in.assign(g.nq, 0);
  g.is_out.assign(g.nq, 0);
  for (int32_t q : ins) g.is_in[dense(q)] = 1;
  for (int32_t q : outs) g.is_out[dense(q)] = 1;
  for (const owqs_cmd &c : cmds) {
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
      g.order.push_back(dense(c.q0));
    }
  }
  for (auto &n : g.nbr) std::sort(n.begin(), n.end());
  return g;
}

// Is there x over GF(2) with  sum_k adj(r, k) x_k = [r == target]  for every
// guarded r?  `guarded(q)` and `candidate(q)` select the two sides.
template <class Guarded, class Candidate>
bool solvable(const OpenGraph &g, int target, const std::vector<int> &guard_list, Guarded guarded,
              Candidate candidate, std::vector<int> &col_of, std::vector<int> &row_of) {
  // columns: candidates adjacent to a guarded qubit; rows: guarded qubits
  // adjacent to a column (the target must be one, or its equation is 0 = 1)
  std::vector<int> cols, rows;
  for (int r : guard_list)
    for (int k : g.nbr[r])
      if (candidate(k) && col_of[k] < 0) {
        col_of[k] = (int)cols.size();
        cols.push_back(k);
      }
  for (int k : cols)
    for (int r : g.nbr[k])
      if (guarded(r) && row_of[r] < 0) {
        row_of[r] = (int)rows.size();
        rows.push_back(r);
      }
  const bool target_in = row_of[target] >= 0;
  bool ok = false;
  if (target_in) {
    const size_t words = (cols.size() + 1 + 63) / 64;  // last bit: right-hand side
    const size_t rhs = cols.size();
    std::vector<uint64_t> m(rows.size() * words, 0);
    for (size_t i = 0; i < rows.size(); ++i) {
      uint64_t *row = &m[i * words];
      for (int k : g.nbr[rows[i]])
        if (col_of[k] >= 0) row[col_of[k] / 64] |= uint64_t(1) << (col_of[k] % 64);
      if (rows[i] == target) row[rhs / 64] |= uint64_t(1) << (rhs % 64);
    }
    // Gaussian elimination; inconsistent iff a row reduces to 0 = 1
    size_t pivot_row = 0;
    for (size_t c = 0; c < cols.size() && pivot_row < rows.size(); ++c) {
      const size_t w = c / 64;
      const uint64_t bit = uint64_t(1) << (c % 64);
      size_t p = pivot_row;
      while (p < rows.size() && !(m[p * words + w] & bit)) ++p;
      if (p == rows.size()) continue;
      if (p != pivot_row)
        for (size_t x = 0; x < words; ++x) std::swap(m[p * words + x], m[pivot_row * words + x]);
      for (size_t r = 0; r < rows.size(); ++r)
        if (r != pivot_row && (m[r * words + w] & bit))
          for (size_t x = 0; x < words; ++x) m[r * words + x] ^= m[pivot_row * words + x];
      ++pivot_row;
    }
    ok = true;
    const uint64_t rbit = uint64_t(1) << (rhs % 64);
    for (size_t r = pivot_row; r < rows.size(); ++r)
      if (m[r * words + rhs / 64] & rbit) ok = false;
  }
  for (int k : cols) col_of[k] = -1;
  for (int r : rows) row_of[r] = -1;
  return ok;
}

}  // namespace
}  // namespace owqs

using namespace owqs;

extern "C" {

owqs_status owqs_pattern_certify(const owqs_pattern *pat, uint8_t *witness, size_t n_meas, int32_t *n_certified,
                                 int32_t *first_missing) {
  if (!pat) return OWQS_E_INVALID_ARG;
  OpenGraph g = graph_of(pat);
  if (witness && n_meas != g.order.size())
    return pattern_fail(pat, OWQS_E_INVALID_ARG, "certify: n_meas must equal the pattern's M count");
  std::vector<int> pos(g.nq, INT32_MAX);  // measurement position; outputs and unmeasured: after all
  for (size_t k = 0; k < g.order.size(); ++k) pos[g.order[k]] = (int)k;
  std::vector<int> col_of(g.nq, -1), row_of(g.nq, -1), guard;
  int32_t count = 0, first = -1;
  for (size_t k = 0; k < g.order.size(); ++k) {
    const int v = g.order[k];
    guard.push_back(v);  // the qubits measured so far, v included
    const int pv = (int)k;
    auto guarded = [&](int q) { return pos[q] <= pv; };
    auto candidate = [&](int q) { return pos[q] > pv && !g.is_in[q]; };
    const bool ok = solvable(g, v, guard, guarded, candidate, col_of, row_of);
    if (witness) witness[k] = ok ? 1 : 0;
    if (ok) ++count;
    else if (first < 0) first = (int32_t)k;
  }
  if (n_certified) *n_certified = count;
  if (first_missing) *first_missing = first;
  return OWQS_OK;
}

owqs_status owqs_pattern_gflow(const owqs_pattern *pat, int32_t *exists, int32_t *depth, int32_t *layer,
                               size_t n_meas) {
  if (!pat) return OWQS_E_INVALID_ARG;
  OpenGraph g = graph_of(pat);
  if (layer && n_meas != g.order.size())
    return pattern_fail(pat, OWQS_E_INVALID_ARG, "gflow: n_meas must equal the pattern's M count");
  std::vector<int> lay(g.nq, -1);  // -1: not added yet
  std::vector<int> pending;        // qubits not added (the measured ones)
  for (int q = 0; q < g.nq; ++q) {
    if (g.is_out[q]) lay[q] = 0;
    else pending.push_back(q);
  }
  std::vector<int> col_of(g.nq, -1), row_of(g.nq, -1);
  int round = 0;
  while (!pending.empty()) {
    ++round;
    auto guarded = [&](int q) { return lay[q] < 0; };
    auto candidate = [&](int q) { return lay[q] >= 0 && !g.is_in[q]; };
    std::vector<int> added;
    for (int u : pending) {
      // only a qubit next to a candidate can be corrected
      bool near = false;
      for (int k : g.nbr[u]) near = near || candidate(k);
      if (near && solvable(g, u, pending, guarded, candidate, col_of, row_of)) added.push_back(u);
    }
    if (added.empty()) break;
    for (int u : added) lay[u] = round;
    std::vector<int> rest;
    for (int u : pending)
      if (lay[u] < 0) rest.push_back(u);
    pending.swap(rest);
  }
  const bool ok = pending.empty();
  if (exists) *exists = ok ? 1 : 0;
  if (depth) *depth = ok ? round : 0;
  if (layer)
    for (size_t k = 0; k < g.order.size(); ++k) layer[k] = lay[g.order[k]] < 0 ? 0 : lay[g.order[k]];
  return OWQS_OK;
}

}  // extern "C"
