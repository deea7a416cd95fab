// owqs_sample_host.cpp -- drawn outcomes (Fig. 6): the sampled plan, the
// per-run tables of drawn windows, the runs, and the C ABI entry points for
// seeded and drawn outcomes.  The kernels are in owqs_sample.hip.
#include "owqs_host_impl.h"

namespace owqs {

// The plan for drawn outcomes: one step per command in execution order (N
// appends the top slot, M moves the top qubit into the measured slot, as in
// compile_plan); every X/Z is kept (its signal is known only on the device)
// and the signal domains become lists of measurement indices.
void compile_sampled(owqs_pattern *p) {
  std::vector<int> slot_of(p->nq, -1), qubit_at(OWQS_MAX_WIDTH + 1, -1), m_of(p->nq, -1);
  int n = (int)p->inputs.size();
  for (int k = 0; k < n; ++k) {
    slot_of[p->inputs[k]] = k;
    qubit_at[k] = p->inputs[k];
  }
  const double r2 = 1.0 / std::sqrt(2.0);
  double pending = 1.0;
  int m = 0;
  p->s_steps.clear();
  p->s_dom.clear();
  p->s_folds.clear();
  auto dom = [&](const std::vector<int> &qs) {
    SigRef r{(int)p->s_dom.size(), (int)qs.size()};
    for (int q : qs) p->s_dom.push_back(m_of[q]);  // D0: measured before
    return r;
  };
  const size_t nc = p->cmds.size();
  for (size_t i = 0; i < nc; ++i) {
    const Cmd &c = p->cmds[i];
    // a window N w; E's on v or w; M v; X/Z on w with an odd number of
    // E(v, w): its outcome has probability exactly 1/2 (w is a fresh |+>
    // neighbour of v), so it is drawn without a probability pass and runs as
    // one 2x2 pass; the corrections on w are resolved on the device
    if (c.op == OWQS_OP_N && i + 2 < nc) {
      const int w = c.q0;
      size_t j = i + 1;
      while (j < nc && p->cmds[j].op == OWQS_OP_E) ++j;
      if (j > i + 1 && j < nc && p->cmds[j].op == OWQS_OP_M && p->cmds[j].q0 != w && slot_of[p->cmds[j].q0] >= 0) {
        const Cmd &mm = p->cmds[j];
        const int v = mm.q0;
        bool ok = true;
        int vw = 0;
        uint64_t mask_b = 0, mask_o1 = 0;
        for (size_t e = i + 1; e < j && ok; ++e) {
          const int a = p->cmds[e].q0, b = p->cmds[e].q1;
          if ((a == v && b == w) || (a == w && b == v)) {
            ++vw;
          } else if (a == v || b == v || a == w || b == w) {
            const int x = (a == v || a == w) ? b : a;
            ok = slot_of[x] >= 0;
            if (ok) {
              if (a == v || b == v) mask_b ^= uint64_t(1) << slot_of[x];
              else mask_o1 ^= uint64_t(1) << slot_of[x];
            }
          } else {
            ok = false;
          }
        }
        if (ok && vw % 2 == 1) {
          owqs_pattern::SStep st{};
          st.kind = S_J;
          st.n = n;
          st.b0 = slot_of[v];
          st.m = m;
          st.alpha = p->angles[m];
          st.host_factor = pending * r2;
          st.s = dom(mm.s);
          st.t = dom(mm.t);
          st.win.mask_b = mask_b;
          st.win.mask_o1 = mask_o1;
          st.win.vw_even = 0;
          m_of[v] = m++;
          st.fold_off = (int)p->s_folds.size();
          size_t q = j + 1;
          while (q < nc && (p->cmds[q].op == OWQS_OP_X || p->cmds[q].op == OWQS_OP_Z) && p->cmds[q].q0 == w) {
            p->s_folds.push_back(FoldRef{p->cmds[q].op == OWQS_OP_X ? 1 : 0, dom(p->cmds[q].s)});
            ++q;
          }
          st.fold_len = (int)p->s_folds.size() - st.fold_off;
          p->s_steps.push_back(st);
          slot_of[w] = slot_of[v];
          qubit_at[slot_of[v]] = w;
          slot_of[v] = -1;
          pending = 1.0;
          i = q - 1;
          continue;
        }
      }
    }
    owqs_pattern::SStep st{};
    st.n = n;
    switch (c.op) {
      case OWQS_OP_N:
        st.kind = S_N;
        slot_of[c.q0] = n;
        qubit_at[n] = c.q0;
        ++n;
        pending *= r2;
        break;
      case OWQS_OP_E:
        st.kind = S_E;
        st.b0 = slot_of[c.q0];
        st.b1 = slot_of[c.q1];
        break;
      case OWQS_OP_X:
      case OWQS_OP_Z:
        st.kind = c.op == OWQS_OP_X ? S_X : S_Z;
        st.b0 = slot_of[c.q0];
        st.s = dom(c.s);
        break;
      case OWQS_OP_M: {
        st.kind = S_M;
        st.b0 = slot_of[c.q0];
        st.m = m;
        st.alpha = p->angles[m];
        st.host_factor = pending;
        st.s = dom(c.s);
        st.t = dom(c.t);
        m_of[c.q0] = m++;
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
        continue;
    }
    p->s_steps.push_back(st);
  }
  // drawn windows have p = 1/2 exactly: like the fused plans (half_prob),
  // they record it without the sum, their FP32 factors chosen with error
  // feedback (rounded_factor), at most kHalfRun in a row
  {
    double e = 1.0;
    int run = 0;
    for (owqs_pattern::SStep &x : p->s_steps) {
      if (x.kind == S_J) {
        x.host_factor = rounded_factor(x.host_factor, e);
        x.half = run + 1 <= p->half_cap;
        run = x.half ? run + 1 : 0;
      } else if (x.kind == S_M) {
        e = 1.0;
        run = 0;
      }
    }
  }
  p->s_final_where.assign(p->outputs.size(), 0);
  for (size_t k = 0; k < p->outputs.size(); ++k) p->s_final_where[k] = slot_of[p->outputs[k]];
  p->s_final_factor = pending;
  p->s_analytic = true;
  for (const owqs_pattern::SStep &x : p->s_steps)
    if (x.kind != S_N && x.kind != S_E && x.kind != S_J) p->s_analytic = false;
  p->s_valid = true;
  p->s_uploaded = false;
  p->a_wins_valid = false;
  if (p->s_exec) { (void)hipGraphExecDestroy(p->s_exec); p->s_exec = nullptr; }
  if (p->s_graph) { (void)hipGraphDestroy(p->s_graph); p->s_graph = nullptr; }
}

SampleMem sample_mem(owqs_pattern *p) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  char *b = static_cast<char *>(p->s_mem);
  const size_t nm = std::max<size_t>(p->n_meas, 1);
  SampleMem sm{};
  sm.u = reinterpret_cast<double *>(b);
  sm.outc = reinterpret_cast<int *>(b + up(nm * sizeof(double)));
  sm.coef = reinterpret_cast<float2 *>(b + up(nm * sizeof(double)) + up(nm * sizeof(int)));
  sm.fold = reinterpret_cast<int *>(b + up(nm * sizeof(double)) + up(nm * sizeof(int)) + 16);
  sm.dom = reinterpret_cast<int *>(b + up(nm * sizeof(double)) + up(nm * sizeof(int)) + 256);
  sm.folds = reinterpret_cast<FoldRef *>(b + up(nm * sizeof(double)) + up(nm * sizeof(int)) + 256 +
                                         up(std::max<size_t>(p->s_dom.size(), 1) * sizeof(int)));
  return sm;
}

hipError_t launch_sampled(owqs_pattern *p, hipStream_t s) {
  const SampleMem sm = sample_mem(p);
  hipError_t e = hipSuccess;
  for (const owqs_pattern::SStep &x : p->s_steps) {
    if (e != hipSuccess) break;
    switch (x.kind) {
      case S_N: e = launch_prepare(p->psi, x.n, s); break;
      case S_E: e = launch_cz(p->psi, x.n, x.b0, x.b1, s); break;
      case S_X:
      case S_Z: e = launch_s_pauli(p->psi, x.n, x.b0, x.kind == S_X, x.s, sm.dom, sm.outc, s); break;
      case S_M: {
        unsigned g = 0, g2 = 0;
        e = launch_s_prob(p->psi, x.n, x.b0, x.alpha, x.s, x.t, sm.dom, sm.outc, p->book.partials, &g, s);
        if (e == hipSuccess)
          e = launch_s_decide(p->book.partials, g, sm.u, x.m, x.alpha, x.s, x.t, sm.dom, sm.outc, sm.coef, s);
        MeasureArgs a{};
        a.coef_dev = sm.coef;
        a.host_factor = x.host_factor;
        a.reduce = kReduceRenorm;
        a.m_index = x.m;
        a.book = p->book;
        if (e == hipSuccess) e = launch_measure(p->psi, x.n, x.b0, a, s, &g2);
        if (e == hipSuccess) e = launch_finish(a, g2, s);
        break;
      }
      case S_J: {
        unsigned g = 0;
        e = launch_s_jdecide(sm.u, x.m, x.alpha, x.s, x.t, sm.dom, sm.outc, sm.coef, sm.folds + x.fold_off, x.fold_len,
                             sm.fold, s);
        MeasureArgs a{};
        a.coef_dev = sm.coef;
        a.fold_dev = sm.fold;
        a.host_factor = x.host_factor;
        a.reduce = x.half ? kReduceNone : kReduceRenorm;  // p = 1/2 exactly: sigma waits for the next sum
        a.prob_half = x.half ? 1 : 0;
        a.m_index = x.m;
        a.book = p->book;
        if (e == hipSuccess) e = launch_jwindow(p->psi, x.n, x.b0, a, x.win, s, &g);
        if (e == hipSuccess) e = launch_finish(a, g, s);
        break;
      }
      default: break;
    }
  }
  return e;
}

// Drawn outcomes when every M is a window with p = 1/2 (s_analytic): each
// outcome is u[m] <= 1/2, known before the run, so the signals, coefficients
// and folded corrections of all windows are resolved at once by one device
// kernel (k_s_resolve) from the uploaded uniforms, and the fused plan (tile
// passes) runs with them from device tables; the run is one graph and needs
// no host synchronisation.  Returns false (nothing done) when the fused plan
// has steps whose form depends on the outcomes (a separate M, X or Z).
bool run_analytic(owqs_pattern *p, const void *input, size_t want, int input_on_device, hipStream_t s,
                  owqs_status &st) {
  st = OWQS_OK;
  if (p->dirty) compile(p);
  for (const Step &x : p->xsteps)
    if (x.kind == S_M || x.kind == S_X || x.kind == S_Z) return false;
  for (const FuseOp &op : p->fuse_ops)
    if (op.kind == DK_X || op.kind == DK_Z) return false;
  const size_t nm = std::max<size_t>(p->n_meas, 1);
  // each window's row in the tile-pass command table (its coefficient and
  // folds are written there by the resolving kernel)
  std::vector<int> fop_of(std::max<size_t>(p->n_meas, 1), -1);
  for (size_t i = 0; i < p->fuse_ops.size(); ++i)
    if (p->fuse_ops[i].kind == DK_J) fop_of[p->fuse_ops[i].m_index] = (int)i;
  std::vector<DrawWin> wins;
  for (const owqs_pattern::SStep &x : p->s_steps)
    if (x.kind == S_J) wins.push_back(DrawWin{x.alpha, x.s, x.t, x.m, x.fold_off, x.fold_len, fop_of[x.m]});
  // the composed maps (their rows are formed again from the resolved windows)
  std::vector<int> moff;
  for (size_t q = 0; q < p->fuse_msrc.size(); q += 2 + size_t(p->fuse_msrc[q + 1])) moff.push_back(int(q));
  const int nmaps = int(moff.size());
  hipError_t e = hipSuccess;
  const size_t cbytes = (nm * sizeof(float2) + 255) & ~size_t(255);
  const size_t fbytes = (3 * nm * sizeof(int) + 255) & ~size_t(255);
  const size_t wbytes = (std::max<size_t>(wins.size(), 1) * sizeof(DrawWin) + 255) & ~size_t(255);
  const size_t mbytes = (p->fuse_msrc.size() + moff.size() + 1) * sizeof(int);
  const size_t need = cbytes + fbytes + wbytes + mbytes;
  if (p->a_cap < need) {
    if (p->a_mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p->a_mem);
    }
    if (p->a_exec) { (void)hipGraphExecDestroy(p->a_exec); p->a_exec = nullptr; }
    if (p->a_graph) { (void)hipGraphDestroy(p->a_graph); p->a_graph = nullptr; }
    p->a_mem = nullptr;
    p->a_cap = 0;
    p->a_wins_valid = false;
    e = hipMalloc(&p->a_mem, need);
    if (e != hipSuccess) { st = fail(p->ctx, OWQS_E_NOMEM, "drawn-window tables"); return true; }
    p->a_cap = need;
  }
  float2 *ctab = static_cast<float2 *>(p->a_mem);
  int *ftab = reinterpret_cast<int *>(static_cast<char *>(p->a_mem) + cbytes);
  DrawWin *dwins = reinterpret_cast<DrawWin *>(static_cast<char *>(p->a_mem) + cbytes + fbytes);
  int *mrefs = reinterpret_cast<int *>(static_cast<char *>(p->a_mem) + cbytes + fbytes + wbytes);
  int *moffs = mrefs + p->fuse_msrc.size();
  if (!p->a_wins_valid) {
    // once per plan (synchronous: a run in flight may still read the table)
    if (p->a_exec) { (void)hipGraphExecDestroy(p->a_exec); p->a_exec = nullptr; }
    if (p->a_graph) { (void)hipGraphDestroy(p->a_graph); p->a_graph = nullptr; }
    e = hipStreamSynchronize(s);
    if (e == hipSuccess && !wins.empty())
      e = hipMemcpy(dwins, wins.data(), wins.size() * sizeof(DrawWin), hipMemcpyHostToDevice);
    if (e == hipSuccess && nmaps > 0)
      e = hipMemcpy(mrefs, p->fuse_msrc.data(), p->fuse_msrc.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && nmaps > 0) e = hipMemcpy(moffs, moff.data(), moff.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) { st = hip_fail(p->ctx, e, "drawn-window table"); return true; }
    p->a_wins_valid = true;
  }
  const SampleMem sm = sample_mem(p);
  // the window rows are rewritten by every drawn run (no upload per run); a
  // forced run uploads the table again
  if (!p->dev_fuse_valid) st = upload_fuse(p);
  if (st != OWQS_OK) return true;
  p->fuse_patched = true;
  FuseOp *const mrows = p->dev_fuse + fuse_mops_base(p->fuse_ops.size(), p->fuse_m.size());
  end_ranged(p);
  const size_t nin = p->inputs.size();
  e = launch_init(p->psi, p->book, s, nin == 0 && input == nullptr ? 1 : 0);
  if (e == hipSuccess && (nin > 0 || input != nullptr))
    e = hipMemcpyAsync(p->psi, input, want * sizeof(float2),
                       input_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
  if (e != hipSuccess) { st = hip_fail(p->ctx, e, "input"); return true; }
  if (p->use_graph && !p->xsteps.empty()) {
    if (!p->a_exec) {
      if (!p->cap_stream) {
        e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) { st = hip_fail(p->ctx, e, "capture stream"); return true; }
      }
      e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) { st = hip_fail(p->ctx, e, "begin capture"); return true; }
      hipError_t le = launch_s_resolve(dwins, (int)wins.size(), sm.u, sm.dom, sm.folds, sm.outc, ctab, ftab,
                                       p->dev_fuse, p->cap_stream);
      if (le == hipSuccess) le = launch_s_compose(p->dev_fuse, mrows, mrefs, moffs, nmaps, p->cap_stream);
      if (le == hipSuccess)
        le = launch_range(p, p->xsteps, 0, p->xsteps.size(), kReduceRenorm, p->cap_stream, nullptr, ctab, ftab,
                          nullptr, nullptr, true);
      e = hipStreamEndCapture(p->cap_stream, &p->a_graph);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->a_exec, p->a_graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (p->a_graph) { (void)hipGraphDestroy(p->a_graph); p->a_graph = nullptr; }
        p->a_exec = nullptr;
        st = hip_fail(p->ctx, e, "graph capture");
        return true;
      }
    }
    e = hipGraphLaunch(p->a_exec, s);
  } else {
    e = launch_s_resolve(dwins, (int)wins.size(), sm.u, sm.dom, sm.folds, sm.outc, ctab, ftab, p->dev_fuse, s);
    if (e == hipSuccess) e = launch_s_compose(p->dev_fuse, mrows, mrefs, moffs, nmaps, s);
    if (e == hipSuccess)
      e = launch_range(p, p->xsteps, 0, p->xsteps.size(), kReduceRenorm, s, nullptr, ctab, ftab, nullptr, nullptr,
                       true);
  }
  if (e != hipSuccess) { st = hip_fail(p->ctx, e, "kernel launch"); return true; }
  p->ran = true;
  p->ss_ran = false;
  p->batch_ran = false;
  p->out_in_order = false;
  p->sampled_ran = true;
  p->an_ran = true;
  p->ran_mode = kReduceRenorm;
  return true;
}

owqs_status run_sampled(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device, void *stream) {
  const size_t nin = p->inputs.size();
  if (owqs_status w = width_guard(p)) return w;
  const size_t want = size_t(1) << nin;
  if (n_amps != want) return fail(p->ctx, OWQS_E_INVALID_ARG, "input size must be 2^(number of inputs)");
  if (nin > 0 && !input) return fail(p->ctx, OWQS_E_INVALID_ARG, "null input");
  if (p->mode != OWQS_MODE_OWQS) return fail(p->ctx, OWQS_E_STATE, "drawn outcomes need OWQS mode (probabilities)");
  owqs_status st = ensure_device(p);
  if (st != OWQS_OK) return st;
  if (!p->s_valid) compile_sampled(p);
  const size_t nm = std::max<size_t>(p->n_meas, 1);
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t need = up(nm * sizeof(double)) + up(nm * sizeof(int)) + 256 +
                      up(std::max<size_t>(p->s_dom.size(), 1) * sizeof(int)) +
                      up(std::max<size_t>(p->s_folds.size(), 1) * sizeof(FoldRef));
  hipError_t e = hipSuccess;
  if (p->s_cap < need) {
    if (p->s_mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p->s_mem);
    }
    p->s_mem = nullptr;
    p->s_cap = 0;
    e = hipMalloc(&p->s_mem, need);
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "sampling tables");
    p->s_cap = need;
    p->s_uploaded = false;
    p->a_wins_valid = false;  // the drawn-window graph reads these tables
    if (p->s_exec) { (void)hipGraphExecDestroy(p->s_exec); p->s_exec = nullptr; }
    if (p->s_graph) { (void)hipGraphDestroy(p->s_graph); p->s_graph = nullptr; }
  }
  const SampleMem sm = sample_mem(p);
  if (!p->s_uploaded) {  // synchronous: the host tables may change after this call
    if (p->n_meas) e = hipMemcpy(sm.u, p->uniforms.data(), p->n_meas * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->s_dom.empty())
      e = hipMemcpy(sm.dom, p->s_dom.data(), p->s_dom.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->s_folds.empty())
      e = hipMemcpy(sm.folds, p->s_folds.data(), p->s_folds.size() * sizeof(FoldRef), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "sampling tables upload");
    p->s_uploaded = true;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->s_analytic && p->exec != OWQS_EXEC_PLAIN) {
    owqs_status ast = OWQS_OK;
    if (run_analytic(p, input, want, input_on_device, s, ast)) return ast;
  }
  end_ranged(p);
  e = launch_init(p->psi, p->book, s, nin == 0 && input == nullptr ? 1 : 0);
  if (e == hipSuccess && (nin > 0 || input != nullptr))
    e = hipMemcpyAsync(p->psi, input, want * sizeof(float2),
                       input_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "input");
  if (p->use_graph && !p->s_steps.empty()) {
    if (!p->s_exec) {
      if (!p->cap_stream) {
        e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "capture stream");
      }
      e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(p->ctx, e, "begin capture");
      hipError_t le = launch_sampled(p, p->cap_stream);
      e = hipStreamEndCapture(p->cap_stream, &p->s_graph);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->s_exec, p->s_graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (p->s_graph) { (void)hipGraphDestroy(p->s_graph); p->s_graph = nullptr; }
        p->s_exec = nullptr;
        return hip_fail(p->ctx, e, "graph capture");
      }
    }
    e = hipGraphLaunch(p->s_exec, s);
  } else {
    e = launch_sampled(p, s);
  }
  if (e != hipSuccess) return hip_fail(p->ctx, e, "kernel launch");
  p->ran = true;
  p->ss_ran = false;
  p->batch_ran = false;
  p->out_in_order = false;
  p->sampled_ran = true;
  p->an_ran = false;
  p->ran_mode = kReduceRenorm;
  return OWQS_OK;
}


}  // namespace owqs

extern "C" {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k (k = 0, 1, ...)
// of the generator started at `seed` is mix(seed + (k + 1) * gamma); the
// outcome of the m-th M is the top bit of output m.
owqs_status owqs_set_outcome_seed(owqs_pattern *p, uint64_t seed) {
  if (!p) return OWQS_E_INVALID_ARG;
  uint64_t x = seed;
  for (int m = 0; m < p->n_meas; ++m) {
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p->outcomes[m] = uint8_t(z >> 63);
  }
  p->dirty = true;
  p->sampling = false;
  return OWQS_OK;
}

owqs_status owqs_get_outcomes(const owqs_pattern *p, uint8_t *bits, size_t n_meas) {
  if (!p || (n_meas && !bits)) return OWQS_E_INVALID_ARG;
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "outcome count != number of M commands");
  std::copy(p->outcomes.begin(), p->outcomes.end(), bits);
  return OWQS_OK;
}

owqs_status owqs_set_uniforms(owqs_pattern *p, const double *u, size_t n_meas) {
  if (!p) return OWQS_E_INVALID_ARG;
  if (!u) {
    if (n_meas) return OWQS_E_INVALID_ARG;
    p->sampling = false;
    return OWQS_OK;
  }
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "uniform count != number of M commands");
  for (size_t k = 0; k < n_meas; ++k)
    if (!(u[k] >= 0.0 && u[k] < 1.0)) return fail(p->ctx, OWQS_E_INVALID_ARG, "uniforms must lie in [0, 1)");
  // a run in flight may still read the device copy: let it finish first
  if (p->s_mem && p->ctx->device >= 0) (void)hipDeviceSynchronize();
  p->uniforms.assign(u, u + n_meas);
  p->sampling = true;
  p->s_uploaded = false;
  return OWQS_OK;
}

owqs_status owqs_read_outcomes(owqs_pattern *p, uint8_t *bits, size_t n_meas, void *stream) {
  if (!p || (n_meas && !bits)) return OWQS_E_INVALID_ARG;
  if (n_meas != (size_t)p->n_meas) return fail(p->ctx, OWQS_E_INVALID_ARG, "outcome count != number of M commands");
  if (!p->sampled_ran) return owqs_get_outcomes(p, bits, n_meas);
  std::vector<int> o(std::max<size_t>(n_meas, 1));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (n_meas) e = hipMemcpyAsync(o.data(), sample_mem(p).outc, n_meas * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "read outcomes");
  for (size_t k = 0; k < n_meas; ++k) bits[k] = uint8_t(o[k] & 1);
  return OWQS_OK;
}


}  // extern "C"
