// owqs_substate_host.cpp -- the sub-state executor (OWQS_EXEC_SUBSTATES,
// Sec. 4.1, Sec. 4.4.1): its plan, its runs and read-out, and its C ABI
// entry points.  The kernels are in owqs_substate.hip.
#include "owqs_host_impl.h"

namespace owqs {

// The launch order of the sub-state plan, with each sub-state's runs of
// window/E/X/Z steps grouped into tile passes as in the single-vector plan.
// Sub-states occupy disjoint regions and scales, so a step of one commutes
// with every step of another: a sub-state's groupable steps are held back
// (in order) until a step of that sub-state that cannot join them, or a merge
// that involves it, and then go out as tile passes, ahead of that step.  The
// order inside each sub-state is the plan's.
void group_substates(owqs_pattern *p) {
  p->ss_run.clear();
  p->ss_groups.clear();
  p->ss_fuse_ops.clear();
  p->ss_fuse_mops.clear();
  p->ss_fuse_m.clear();
  p->ss_dev_fuse_valid = false;
  const size_t nch = p->ss_chains.size();
  std::vector<std::vector<int>> held(nch);
  auto groupable = [](int k) { return k == SS_J || k == SS_E || k == SS_X || k == SS_Z; };
  auto flush = [&](int c) {
    std::vector<int> &h = held[c];
    if (h.empty()) return;
    std::vector<Step> run;
    for (int i : h) {
      const SubStep &x = p->ss_steps[i];
      Step st{};
      st.kind = x.kind == SS_J ? S_J : x.kind == SS_E ? S_E : x.kind == SS_X ? S_X : S_Z;
      st.n = x.n;
      st.b0 = x.b0;
      st.b1 = x.b1;
      st.coef = x.coef;
      st.host_factor = x.host_factor;
      st.m_index = x.m_index;
      st.win = x.win;
      st.group = i;  // a step left ungrouped keeps its plan index here
      run.push_back(st);
    }
    std::vector<Step> out;
    group_steps(run, p->mode, p->tile_bits, out, p->ss_groups, p->ss_fuse_ops, p->ss_fuse_m, false,
                &p->ss_fuse_mops);
    for (const Step &x : out)
      p->ss_run.push_back(x.kind == S_F ? SubRun{-1, x.group, c} : SubRun{x.group, -1, c});
    h.clear();
  };
  for (size_t i = 0; i < p->ss_steps.size(); ++i) {
    const SubStep &x = p->ss_steps[i];
    std::vector<int> &h = held[x.chain];
    if (groupable(x.kind) && x.n >= kTileMinWidth) {
      if (!h.empty() && p->ss_steps[h.front()].n != x.n) flush(x.chain);
      h.push_back((int)i);
      continue;
    }
    flush(x.chain);
    if (x.kind == SS_KRON) flush(x.top);
    p->ss_run.push_back(SubRun{(int)i, -1, x.chain});
  }
  for (size_t c = 0; c < nch; ++c) flush((int)c);
  // windows with p = 1/2 that skip their reduction, at most kHalfRun in a
  // row per sub-state (mark_half); a merged sub-state inherits both runs
  std::vector<int> run(nch, 0);
  for (const SubRun &r : p->ss_run) {
    if (r.group >= 0) {
      TileGroup &tg = p->ss_groups[r.group];
      if (tg.ta.nwin == 0) continue;
      tg.half = p->mode == OWQS_MODE_OWQS && tg.half && run[r.chain] + tg.ta.nwin <= p->half_cap;
      run[r.chain] = tg.half ? run[r.chain] + tg.ta.nwin : 0;
      continue;
    }
    SubStep &x = p->ss_steps[r.step];
    if (x.kind == SS_M) {
      run[r.chain] = 0;
    } else if (x.kind == SS_J) {
      x.half = p->mode == OWQS_MODE_OWQS && !x.win.vw_even && run[r.chain] + 1 <= p->half_cap;
      run[r.chain] = x.half ? run[r.chain] + 1 : 0;
    } else if (x.kind == SS_KRON) {
      run[r.chain] += run[x.top];
    }
  }
}

// Sub-state plan (Sec. 4.1, Sec. 4.4.1): every input factor starts as a
// sub-state; N makes a fresh |+> qubit that stays implicit until a command
// touches it; E with a fresh qubit appends it to the other qubit's sub-state
// (a prepare step, as in the single-vector plan), E across two sub-states
// merges them (SS_KRON, the wider one is the base and keeps its region), and
// M eliminates its qubit inside its sub-state (the top qubit moves into the
// freed slot).  Each sub-state keeps its own host factor and FP64 scale.
void compile_substates(owqs_pattern *p) {
  p->ss_steps.clear();
  p->ss_chains.clear();
  p->ss_factors.clear();
  p->ss_vanished.clear();
  const int nq = p->nq;
  std::vector<int> chain_of(nq, -1), slot_of(nq, -1), outcome_of(nq, 0);
  std::vector<char> fresh(nq, 0);
  std::vector<SubChain> &ch = p->ss_chains;
  const double r2 = 1.0 / std::sqrt(2.0);
  auto widen = [&](int c) { ch[c].maxw = std::max(ch[c].maxw, (int)ch[c].at.size()); };
  // input factors
  std::vector<int32_t> nqs = p->ss_in_nq;
  if (nqs.empty() && !p->inputs.empty()) nqs.push_back((int32_t)p->inputs.size());
  size_t off = 0;
  for (int32_t k : nqs) {
    ch.emplace_back();
    const int c = (int)ch.size() - 1;
    for (int32_t j = 0; j < k; ++j) {
      const int q = p->inputs[off + j];
      chain_of[q] = c;
      slot_of[q] = j;
      ch[c].at.push_back(q);
    }
    off += (size_t)k;
    widen(c);
  }
  auto emit = [&](int kind, int c) -> SubStep & {
    SubStep st{};
    st.kind = kind;
    st.chain = c;
    st.n = (int)ch[c].at.size();
    p->ss_steps.push_back(st);
    return p->ss_steps.back();
  };
  auto prep = [&](int c, int q) {
    emit(SS_N, c);
    slot_of[q] = (int)ch[c].at.size();
    chain_of[q] = c;
    fresh[q] = 0;
    ch[c].at.push_back(q);
    ch[c].pend *= r2;
    widen(c);
  };
  auto materialize = [&](int q) {
    ch.emplace_back();
    const int c = (int)ch.size() - 1;
    emit(SS_INIT, c);
    prep(c, q);
    return c;
  };
  int m = 0;
  auto m_coef = [&](const Cmd &c, int mi, int &o) {
    const int sgn = signal(c.s, outcome_of), t = signal(c.t, outcome_of);
    const double theta = (sgn ? -p->angles[mi] : p->angles[mi]) + (t ? M_PI : 0.0);  // Eq. 2
    o = p->outcomes[mi] & 1;
    double cr = std::cos(theta), ci = -std::sin(theta);  // (-1)^o e^{-i theta}  (Eqs. 11-12)
    if (o) { cr = -cr; ci = -ci; }
    return make_float2((float)cr, (float)ci);
  };
  const size_t nc = p->cmds.size();
  for (size_t i = 0; i < nc; ++i) {
    const Cmd &c = p->cmds[i];
    // the window N w; E's on v or w; M v; X/Z on w as one 2x2 pass inside v's
    // sub-state (as in the single-vector plan), when every E partner already
    // sits in v's sub-state
    if (c.op == OWQS_OP_N && i + 2 < nc) {
      const int w = c.q0;
      size_t j = i + 1;
      while (j < nc && p->cmds[j].op == OWQS_OP_E) ++j;
      if (j > i + 1 && j < nc && p->cmds[j].op == OWQS_OP_M && p->cmds[j].q0 != w && !fresh[p->cmds[j].q0] &&
          chain_of[p->cmds[j].q0] >= 0) {
        const Cmd &mm = p->cmds[j];
        const int v = mm.q0, k = chain_of[v];
        bool ok = true;
        int vw = 0;
        uint64_t mask_b = 0, mask_o1 = 0;
        for (size_t e = i + 1; e < j && ok; ++e) {
          const int a = p->cmds[e].q0, b = p->cmds[e].q1;
          if ((a == v && b == w) || (a == w && b == v)) {
            ++vw;
          } else if (a == v || b == v || a == w || b == w) {
            const int x = (a == v || a == w) ? b : a;
            ok = chain_of[x] == k;
            if (ok) {
              if (a == v || b == v) mask_b ^= uint64_t(1) << slot_of[x];
              else mask_o1 ^= uint64_t(1) << slot_of[x];
            }
          } else {
            ok = false;  // an E on two other qubits ends the window
          }
        }
        if (ok && vw > 0) {
          int o = 0;
          SubStep &st = emit(SS_J, k);
          st.b0 = slot_of[v];
          st.coef = m_coef(mm, m, o);
          st.host_factor = ch[k].pend * r2;
          st.m_index = m;
          st.win.mask_b = mask_b;
          st.win.mask_o1 = mask_o1;
          st.win.vw_even = (vw % 2 == 0) ? 1 : 0;
          outcome_of[v] = o;
          ++m;
          ch[k].pend = 1.0;
          int idx[2] = {0, 1}, sgn[2] = {1, 1};
          size_t q = j + 1;
          while (q < nc && (p->cmds[q].op == OWQS_OP_X || p->cmds[q].op == OWQS_OP_Z) && p->cmds[q].q0 == w) {
            if (signal(p->cmds[q].s, outcome_of)) {
              if (p->cmds[q].op == OWQS_OP_X) {
                std::swap(idx[0], idx[1]);
                std::swap(sgn[0], sgn[1]);
              } else {
                sgn[1] = -sgn[1];
              }
            }
            ++q;
          }
          st.win.swap = idx[0] == 1;
          st.win.neg0 = sgn[0] < 0;
          st.win.neg1 = sgn[1] < 0;
          // w takes v's slot
          slot_of[w] = slot_of[v];
          chain_of[w] = k;
          fresh[w] = 0;
          ch[k].at[slot_of[v]] = w;
          chain_of[v] = -1;
          slot_of[v] = -1;
          i = q - 1;
          continue;
        }
      }
    }
    switch (c.op) {
      case OWQS_OP_N:
        fresh[c.q0] = 1;
        break;
      case OWQS_OP_E: {
        const int u = c.q0, v = c.q1;
        if (fresh[u] && fresh[v]) {
          prep(materialize(u), v);
        } else if (fresh[u]) {
          prep(chain_of[v], u);
        } else if (fresh[v]) {
          prep(chain_of[u], v);
        } else if (chain_of[u] != chain_of[v]) {
          int a = chain_of[u], b = chain_of[v];
          if (ch[b].at.size() > ch[a].at.size() || (ch[b].at.size() == ch[a].at.size() && b < a)) std::swap(a, b);
          SubStep &st = emit(SS_KRON, a);
          st.top = b;
          st.top_n = (int)ch[b].at.size();
          const int base_n = (int)ch[a].at.size();
          for (size_t j = 0; j < ch[b].at.size(); ++j) {
            const int q = ch[b].at[j];
            chain_of[q] = a;
            slot_of[q] = base_n + (int)j;
            ch[a].at.push_back(q);
          }
          ch[a].pend *= ch[b].pend;
          ch[b].at.clear();
          ch[b].merged = true;
          widen(a);
        }
        SubStep &st = emit(SS_E, chain_of[u]);
        st.b0 = slot_of[u];
        st.b1 = slot_of[v];
        break;
      }
      case OWQS_OP_X:
      case OWQS_OP_Z: {
        if (!signal(c.s, outcome_of)) break;
        if (fresh[c.q0]) materialize(c.q0);
        SubStep &st = emit(c.op == OWQS_OP_X ? SS_X : SS_Z, chain_of[c.q0]);
        st.b0 = slot_of[c.q0];
        break;
      }
      case OWQS_OP_M: {
        const int q = c.q0;
        if (fresh[q]) materialize(q);
        const int k = chain_of[q];
        int o = 0;
        const float2 cf = m_coef(c, m, o);
        SubStep &st = emit(SS_M, k);
        st.b0 = slot_of[q];
        st.coef = cf;
        st.host_factor = ch[k].pend;
        st.m_index = m;
        ch[k].pend = 1.0;
        outcome_of[q] = o;
        ++m;
        std::vector<int> &at = ch[k].at;
        const int top = at.back();
        if (top != q) {
          at[slot_of[q]] = top;
          slot_of[top] = slot_of[q];
        }
        at.pop_back();
        chain_of[q] = -1;
        slot_of[q] = -1;
        break;
      }
      default:
        break;
    }
  }
  for (int q : p->outputs)
    if (fresh[q]) materialize(q);
  // read-out factors, ordered by their first output; vanished sub-states
  std::vector<int> pos(nq, -1);
  for (size_t k = 0; k < p->outputs.size(); ++k) pos[p->outputs[k]] = (int)k;
  std::vector<int> factor_of(ch.size(), -1);
  for (size_t k = 0; k < p->outputs.size(); ++k) {
    const int q = p->outputs[k], c = chain_of[q];
    if (factor_of[c] < 0) {
      factor_of[c] = (int)p->ss_factors.size();
      SubFactor f{};
      f.chain = c;
      p->ss_factors.push_back(f);
    }
    SubFactor &f = p->ss_factors[factor_of[c]];
    f.qubits.push_back(q);
    f.where.push_back(slot_of[q]);
    f.mask |= uint64_t(1) << k;
  }
  for (size_t c = 0; c < ch.size(); ++c)
    if (!ch[c].merged && ch[c].at.empty()) p->ss_vanished.push_back((int)c);
  p->ss_width = 0;
  for (const SubChain &c : ch) p->ss_width = std::max(p->ss_width, c.maxw);
  // every step stays inside its sub-state's region (checked before any launch)
  p->ss_plan_ok = true;
  for (const SubStep &x : p->ss_steps) {
    const int w = ch[x.chain].maxw;
    bool ok = x.n <= w;
    switch (x.kind) {
      case SS_N: ok = ok && x.n + 1 <= w; break;
      case SS_E: ok = ok && x.b0 >= 0 && x.b1 >= 0 && x.b0 < x.n && x.b1 < x.n && x.b0 != x.b1; break;
      case SS_X:
      case SS_Z:
      case SS_M:
      case SS_J: ok = ok && x.b0 >= 0 && x.b0 < x.n; break;
      case SS_KRON:
        ok = ok && x.top != x.chain && x.n >= 1 && x.top_n >= 1 && x.n + x.top_n <= w &&
             x.top_n <= ch[x.top].maxw;
        break;
      default: break;
    }
    if (!ok) p->ss_plan_ok = false;
  }
  if (p->mode == OWQS_MODE_OWQS) {  // FP32 factors of p = 1/2 windows with error feedback (rounded_factor)
    std::vector<double> e(ch.size(), 1.0);
    for (SubStep &x : p->ss_steps) {
      if (x.kind == SS_J && !x.win.vw_even) x.host_factor = rounded_factor(x.host_factor, e[x.chain]);
      else if (x.kind == SS_M || x.kind == SS_J) e[x.chain] = 1.0;
      else if (x.kind == SS_KRON) e[x.chain] *= e[x.top];
    }
  }
  group_substates(p);
  p->ss_arena = 0;
  if (p->ss_width <= OWQS_MAX_WIDTH) {
    for (SubChain &c : ch) {
      c.off = p->ss_arena;
      const size_t amps = std::max<size_t>(size_t(1) << c.maxw, 4);
      p->ss_arena += (amps + 63) / 64 * 64;  // 512-byte aligned regions
    }
  }
}

void drop_ss_graph(owqs_pattern *p) {
  if (p->ss_exec || p->ss_graph) (void)hipDeviceSynchronize();
  if (p->ss_exec) { (void)hipGraphExecDestroy(p->ss_exec); p->ss_exec = nullptr; }
  if (p->ss_graph) { (void)hipGraphDestroy(p->ss_graph); p->ss_graph = nullptr; }
}


// ---------------------------------------------------------------------------
// sub-state executor runs
// ---------------------------------------------------------------------------
// Launch the plan in ss_run order.  With `ev`: ev[2i] before entry i's main
// kernel, ev[2i+1] after it, ev[2i+2] after the entry (its FP64 finishing
// kernel, if any).
hipError_t launch_substeps(owqs_pattern *p, int reduce, hipStream_t s, std::vector<hipEvent_t> *ev = nullptr) {
  hipError_t e = launch_sub_start(p->ss_sigma, (int)p->ss_chains.size(), p->book.err, s);
  if (ev && e == hipSuccess) e = hipEventRecord((*ev)[0], s);
  for (size_t i = 0; i < p->ss_run.size() && e == hipSuccess; ++i) {
    const SubRun &r = p->ss_run[i];
    if (ev && i > 0) e = hipEventRecord((*ev)[2 * i], s);
    if (e != hipSuccess) break;
    float2 *psi = p->ss_mem + p->ss_chains[r.chain].off;
    MeasureArgs a{};
    a.reduce = reduce;
    a.book = p->book;
    a.book.sigma = p->ss_sigma + r.chain;
    unsigned grid = 0;
    if (r.group >= 0) {  // a tile pass on this sub-state's region, with its scale
      const TileGroup &tg = p->ss_groups[r.group];
      const int *m_of = reinterpret_cast<const int *>(p->ss_dev_fuse + p->ss_fuse_ops.size()) + tg.m_off;
      TileArgs ta = tg.ta;
      if (reduce == kReduceRenorm && tg.half) {  // every window has p = 1/2 exactly
        a.reduce = kReduceNone;
        ta.half_m = m_of;
      }
      const FuseOp *ops = p->ss_dev_fuse + tg.op_off;
      if (tg.mnops > 0 && a.reduce == kReduceNone) {  // no window sums: the composed commands
        ops = p->ss_dev_fuse + fuse_mops_base(p->ss_fuse_ops.size(), p->ss_fuse_m.size()) + tg.mop_off;
        ta.nops = tg.mnops;
        ta.maps = 1;
      }
      e = launch_tile(psi, ta, ops, a, s, &grid);
      if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 1], s);
      if (e == hipSuccess) e = launch_finish_group(a, m_of, tg.ta.nwin, grid, s);
      if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 2], s);
      continue;
    }
    const SubStep &x = p->ss_steps[r.step];
    switch (x.kind) {
      case SS_INIT: e = launch_sub_init(psi, s); break;
      case SS_N: e = launch_prepare(psi, x.n, s); break;
      case SS_E: e = launch_cz(psi, x.n, x.b0, x.b1, s); break;
      case SS_X: e = launch_pauli_x(psi, x.n, x.b0, s); break;
      case SS_Z: e = launch_pauli_z(psi, x.n, x.b0, s); break;
      case SS_KRON:
        e = launch_kron(psi, x.n, p->ss_mem + p->ss_chains[x.top].off, x.top_n, p->ss_sigma + x.chain,
                        p->ss_sigma + x.top, s);
        break;
      case SS_M:
      case SS_J: {
        a.coef = x.coef;
        a.host_factor = x.host_factor;
        a.m_index = x.m_index;
        if (reduce == kReduceRenorm && x.kind == SS_J && x.half) {  // p = 1/2 exactly (see half_prob)
          a.reduce = kReduceNone;
          a.prob_half = 1;
        }
        e = x.kind == SS_M ? launch_measure(psi, x.n, x.b0, a, s, &grid)
                           : launch_jwindow(psi, x.n, x.b0, a, x.win, s, &grid);
        if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 1], s);
        if (e == hipSuccess) e = launch_finish(a, grid, s);
        break;
      }
      default: break;
    }
    if (ev && x.kind != SS_M && x.kind != SS_J && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 1], s);
    if (ev && e == hipSuccess) e = hipEventRecord((*ev)[2 * i + 2], s);
  }
  return e;
}

// Algorithmic bytes of one sub-state step (element level, complex64).
double substep_bytes(const SubStep &x) {
  const double a = std::ldexp(8.0, x.n);
  switch (x.kind) {
    case SS_N: return 2.0 * a;
    case SS_E: return 0.5 * a;
    case SS_M: return 1.5 * a;
    case SS_X: return 2.0 * a;
    case SS_Z: return 1.0 * a;
    case SS_KRON: return a + std::ldexp(8.0, x.top_n) + std::ldexp(8.0, x.n + x.top_n);
    case SS_J: return 2.0 * a;
  }
  return 0.0;
}

bool substates(const owqs_pattern *p) { return p->exec == OWQS_EXEC_SUBSTATES; }

owqs_status refuse_substates(owqs_pattern *p, const char *what) {
  return fail(p->ctx, OWQS_E_STATE, std::string(what) + " does not run the sub-state executor (OWQS_EXEC_SUBSTATES)");
}

// Input factor k (2^nqs[k] complex64) holds the next nqs[k] inputs.
owqs_status run_substates(owqs_pattern *p, const void *const *factors, const int32_t *nqs, size_t nf,
                          int on_device, void *stream, Profile *prof) {
  if (nf && (!factors || !nqs)) return fail(p->ctx, OWQS_E_INVALID_ARG, "null input factors");
  size_t total = 0;
  for (size_t k = 0; k < nf; ++k) {
    if (nqs[k] < 1 || nqs[k] > OWQS_MAX_WIDTH || !factors[k])
      return fail(p->ctx, OWQS_E_INVALID_ARG, "input factor with no qubits, too many, or no data");
    total += (size_t)nqs[k];
  }
  if (total != p->inputs.size()) return fail(p->ctx, OWQS_E_INVALID_ARG, "input factors must cover the inputs");
  std::vector<int32_t> want(nqs, nqs + nf);
  if (nf == 1) want.clear();  // one factor is the default plan
  if (want != p->ss_in_nq) {
    p->ss_in_nq = want;
    p->dirty = true;
  }
  if (p->sampling) return fail(p->ctx, OWQS_E_STATE, "drawn outcomes do not run the sub-state executor");
  owqs_status st = ensure_device(p, false);  // compiles the sub-state plan and checks its width
  if (st != OWQS_OK) return st;
  if (p->dirty) compile(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  const size_t arena = std::max<size_t>(p->ss_arena, 64);
  if (p->ss_mem_cap < arena) {
    drop_ss_graph(p);
    if (p->ss_mem) (void)hipFree(p->ss_mem);
    p->ss_mem = nullptr;
    p->ss_mem_cap = 0;
    e = hipMalloc(&p->ss_mem, arena * sizeof(float2));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, std::string("sub-state arena: ") + hipGetErrorString(e));
    p->ss_mem_cap = arena;
  }
  if (p->ss_sigma_cap < std::max<size_t>(p->ss_chains.size(), 1)) {
    drop_ss_graph(p);
    if (p->ss_sigma) (void)hipFree(p->ss_sigma);
    p->ss_sigma = nullptr;
    p->ss_sigma_cap = 0;
    const size_t n = std::max<size_t>(p->ss_chains.size(), 1);
    e = hipMalloc(&p->ss_sigma, n * sizeof(double));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "sub-state scales");
    p->ss_sigma_cap = n;
  }
  if (!p->ss_dev_fuse_valid) {  // before any capture: the graph holds the table's address
    drop_ss_graph(p);
    st = upload_fuse_table(p->ctx, p->ss_fuse_ops, p->ss_fuse_m, p->ss_dev_fuse, p->ss_dev_fuse_cap,
                           &p->ss_fuse_mops);
    if (st != OWQS_OK) return st;
    p->ss_dev_fuse_valid = true;
  }
  end_ranged(p);
  p->sampled_ran = false;
  p->ran = false;
  p->ss_ran = false;
  for (size_t k = 0; k < nf; ++k) {
    e = hipMemcpyAsync(p->ss_mem + p->ss_chains[k].off, factors[k], (size_t(1) << nqs[k]) * sizeof(float2),
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "input copy");
  }
  const int reduce = p->mode == OWQS_MODE_OWQS ? kReduceRenorm
                     : p->mode == OWQS_MODE_EOWQS_CHECK ? kReduceCheck
                                                        : kReduceNone;
  std::vector<hipEvent_t> ev;
  if (prof) {
    ev.resize(2 * p->ss_run.size() + 1);
    for (auto &x : ev) {
      e = hipEventCreate(&x);
      if (e != hipSuccess) return hip_fail(p->ctx, e, "event");
    }
    e = launch_substeps(p, reduce, s, &ev);
  } else if (p->use_graph) {
    if (p->ss_exec && p->ss_graph_reduce != reduce) drop_ss_graph(p);
    if (!p->ss_exec) {
      if (!p->cap_stream) {
        e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "capture stream");
      }
      e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(p->ctx, e, "begin capture");
      hipError_t le = launch_substeps(p, reduce, p->cap_stream);
      e = hipStreamEndCapture(p->cap_stream, &p->ss_graph);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->ss_exec, p->ss_graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (p->ss_graph) { (void)hipGraphDestroy(p->ss_graph); p->ss_graph = nullptr; }
        p->ss_exec = nullptr;
        return hip_fail(p->ctx, e, "graph capture");
      }
      p->ss_graph_reduce = reduce;
    }
    e = hipGraphLaunch(p->ss_exec, s);
  } else {
    e = launch_substeps(p, reduce, s);
  }
  if (e != hipSuccess) {
    for (auto &x : ev) (void)hipEventDestroy(x);
    return hip_fail(p->ctx, e, "kernel launch");
  }
  p->ran = true;
  p->ss_ran = true;
  p->batch_ran = false;
  p->out_in_order = false;
  p->ran_mode = reduce;
  if (prof) {
    static const int kind_of[] = {-1, OWQS_KIND_N, OWQS_KIND_E, OWQS_KIND_X, OWQS_KIND_Z, OWQS_KIND_M,
                                  OWQS_KIND_KRON, OWQS_KIND_J};
    e = hipStreamSynchronize(s);
    for (size_t i = 0; i < p->ss_run.size() && e == hipSuccess; ++i) {
      const SubRun &r = p->ss_run[i];
      float t = 0.f, f = 0.f;
      e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&f, ev[2 * i + 1], ev[2 * i + 2]);
      if (r.group >= 0) {
        const TileGroup &tg = p->ss_groups[r.group];
        prof->counts[OWQS_KIND_TILE] += 1;
        prof->ms[OWQS_KIND_TILE] += t;
        prof->bytes[OWQS_KIND_TILE] += std::ldexp(16.0, tg.ta.n);  // one read and one write
        if (reduce != kReduceNone && !(reduce == kReduceRenorm && tg.half) && tg.ta.nwin > 0) {
          prof->counts[OWQS_KIND_FINISH] += 1;
          prof->ms[OWQS_KIND_FINISH] += f;
        }
        continue;
      }
      const SubStep &x = p->ss_steps[r.step];
      const int k = kind_of[x.kind];
      if (k < 0) continue;  // a new sub-state's scalar 1
      prof->counts[k] += 1;
      prof->ms[k] += t;
      prof->bytes[k] += substep_bytes(x);
      const bool half = reduce == kReduceRenorm && x.kind == SS_J && x.half;
      if ((x.kind == SS_M || x.kind == SS_J) && reduce != kReduceNone && !half) {
        prof->counts[OWQS_KIND_FINISH] += 1;
        prof->ms[OWQS_KIND_FINISH] += f;
      }
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "profile events");
  }
  return OWQS_OK;
}

// Read every factor (scaled, its qubits in output order) and the scalar of
// the vanished sub-states into ss_stage: factor f at offs[f], the scalar at
// offs.back().
owqs_status stage_substates(owqs_pattern *p, hipStream_t s, std::vector<uint64_t> &offs) {
  offs.clear();
  uint64_t at = 0;
  for (const SubFactor &f : p->ss_factors) {
    offs.push_back(at);
    at += uint64_t(1) << f.qubits.size();
  }
  offs.push_back(at);
  const size_t need = at + std::max<size_t>(p->ss_vanished.size(), 1);
  hipError_t e = hipSuccess;
  if (p->ss_stage_cap < need) {
    if (p->ss_stage) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(p->ss_stage);
    }
    p->ss_stage = nullptr;
    p->ss_stage_cap = 0;
    e = hipMalloc(&p->ss_stage, need * sizeof(float2));
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "sub-state read-out buffer");
    p->ss_stage_cap = need;
  }
  const bool renorm = p->ran_mode == kReduceRenorm;
  for (size_t k = 0; k < p->ss_factors.size() && e == hipSuccess; ++k) {
    const SubFactor &f = p->ss_factors[k];
    const SubChain &c = p->ss_chains[f.chain];
    e = launch_read(p->ss_mem + c.off, p->ss_stage + offs[k], (int)f.qubits.size(), f.where.data(), c.pend,
                    renorm ? p->ss_sigma + f.chain : nullptr, s);
  }
  for (size_t k = 0; k < p->ss_vanished.size() && e == hipSuccess; ++k) {
    const int v = p->ss_vanished[k];
    const SubChain &c = p->ss_chains[v];
    e = launch_read(p->ss_mem + c.off, p->ss_stage + offs.back() + k, 0, nullptr, c.pend,
                    renorm ? p->ss_sigma + v : nullptr, s);
  }
  if (e == hipSuccess) e = launch_cprod(p->ss_stage + offs.back(), (int)p->ss_vanished.size(), s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "sub-state read");
  return OWQS_OK;
}


}  // namespace owqs

extern "C" {

owqs_status owqs_set_input_factors(owqs_pattern *p, const int32_t *factor_nq, size_t nfactors) {
  if (!p || (nfactors && !factor_nq)) return OWQS_E_INVALID_ARG;
  size_t total = 0;
  for (size_t k = 0; k < nfactors; ++k) {
    if (factor_nq[k] < 1 || factor_nq[k] > OWQS_MAX_WIDTH)
      return fail(p->ctx, OWQS_E_INVALID_ARG, "an input factor holds 1 .. OWQS_MAX_WIDTH qubits");
    total += (size_t)factor_nq[k];
  }
  if (nfactors && total != p->inputs.size())
    return fail(p->ctx, OWQS_E_INVALID_ARG, "input factors must cover the inputs");
  std::vector<int32_t> want(factor_nq, factor_nq + nfactors);
  if (nfactors == 1) want.clear();
  if (want != p->ss_in_nq) {
    p->ss_in_nq = want;
    if (substates(p)) p->dirty = true;
  }
  return OWQS_OK;
}

owqs_status owqs_run_factors(owqs_pattern *p, const void *const *factors, const int32_t *factor_nq, size_t nfactors,
                             int input_on_device, void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (!substates(p)) return fail(p->ctx, OWQS_E_STATE, "input factors need the sub-state executor (OWQS_EXEC_SUBSTATES)");
  return run_substates(p, factors, factor_nq, nfactors, input_on_device, stream);
}

owqs_status owqs_read_substates(owqs_pattern *p, void *out_c64, size_t amp_cap, int32_t *factor_nq, int32_t *qubits,
                                size_t factor_cap, int32_t *n_factors, size_t *n_amps, void *scalar_c64,
                                void *stream) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (!p->ss_ran) return fail(p->ctx, OWQS_E_STATE, "the last run did not use the sub-state executor");
  size_t amps = 0;
  for (const SubFactor &f : p->ss_factors) amps += size_t(1) << f.qubits.size();
  if (n_factors) *n_factors = (int32_t)p->ss_factors.size();
  if (n_amps) *n_amps = amps;
  if (factor_nq || qubits) {
    if (factor_cap < p->ss_factors.size()) return fail(p->ctx, OWQS_E_INVALID_ARG, "factor arrays too small");
    size_t k = 0;
    for (size_t f = 0; f < p->ss_factors.size(); ++f) {
      if (factor_nq) factor_nq[f] = (int32_t)p->ss_factors[f].qubits.size();
      for (int q : p->ss_factors[f].qubits)
        if (qubits) qubits[k++] = p->user_id[q];
    }
  }
  if (!out_c64 && !scalar_c64) return OWQS_OK;
  if (out_c64 && amp_cap < amps) return fail(p->ctx, OWQS_E_INVALID_ARG, "amplitude buffer too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<uint64_t> offs;
  owqs_status st = stage_substates(p, s, offs);
  if (st != OWQS_OK) return st;
  hipError_t e = hipSuccess;
  if (out_c64 && amps) e = hipMemcpyAsync(out_c64, p->ss_stage, amps * sizeof(float2), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && scalar_c64)
    e = hipMemcpyAsync(scalar_c64, p->ss_stage + offs.back(), sizeof(float2), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "sub-state read");
  return owqs_check(p, stream);
}


}  // extern "C"
