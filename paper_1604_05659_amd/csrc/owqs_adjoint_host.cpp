// owqs_adjoint_host.cpp -- owqs_adjoint: the batched forward sweep with
// checkpoints and the reversing (or recomputing) backward sweep that gives
// d loss / d alpha.  The kernels are in owqs_adjoint.hip and owqs_tile.hip.
#include "owqs_host_impl.h"

extern "C" {

owqs_status owqs_adjoint(owqs_pattern *p, const void *input_c64, const double *alpha, size_t batch,
                         const int32_t *obs, int32_t nobs, double *loss, double *grad, int32_t ckpt_stride,
                         void *stream) {
  if (!p || !alpha || !loss || !grad || batch == 0 || (nobs && !obs) || nobs < 0)
    return fail(p ? p->ctx : nullptr, OWQS_E_INVALID_ARG, "null pointer or bad size");
  if (batch > 65535) return fail(p->ctx, OWQS_E_INVALID_ARG, "batch above 65535");
  if (substates(p)) return refuse_substates(p, "owqs_adjoint");
  if (!p->inputs.empty() && !input_c64) return fail(p->ctx, OWQS_E_INVALID_ARG, "the pattern needs an input state");
  for (int32_t k = 0; k < nobs; ++k)
    if (obs[k] < 0 || obs[k] >= (int32_t)p->outputs.size())
      return fail(p->ctx, OWQS_E_INVALID_ARG, "observable index outside the outputs");
  owqs_status st = ensure_device(p, false);
  if (st != OWQS_OK) return st;
  end_ranged(p);
  if (p->exec == OWQS_EXEC_PLAIN) {
    p->exec = OWQS_EXEC_AUTO;
    p->dirty = true;
  }
  if (p->dirty) compile(p);
  // structure: a prefix without measurements, then windows and E/X/Z steps
  const size_t ns = p->steps.size();
  size_t fw = ns;
  for (size_t i = 0; i < ns; ++i) {
    if (p->steps[i].kind == S_J) { fw = i; break; }
    if (p->steps[i].kind == S_M)
      return fail(p->ctx, OWQS_E_STATE, "adjoint: a measurement outside an N-E-M window comes before the first window");
  }
  std::vector<size_t> wins;
  for (size_t i = fw; i < ns; ++i) {
    const int k = p->steps[i].kind;
    if (k == S_J) wins.push_back(i);
    else if (k == S_N || k == S_M)
      return fail(p->ctx, OWQS_E_STATE, "adjoint: only windows and E/X/Z steps may follow the first window");
  }
  const int nw = fw < ns ? p->steps[fw].n : p->plan_width;
  const int W = p->plan_width;
  const size_t stride = size_t(1) << W;
  const size_t nwin = wins.size();
  const int cs = ckpt_stride != 0 ? (ckpt_stride > 0 ? ckpt_stride : -ckpt_stride) : 16;
  const size_t nseg = nwin ? (nwin + cs - 1) / cs : 0;
  const unsigned nblk = adj_blocks(nw);
  const unsigned lblk = loss_blocks((int)p->outputs.size());
  // windows with an odd number of E between their two qubits are invertible:
  // the reverse sweep then recovers each window's input from its output
  // (no forward recompute, no stash), restarting from the forward checkpoint
  // at every segment so that rounding cannot build up over more than one
  bool reversible = ckpt_stride >= 0;  // a negative stride asks for the recompute sweep
  for (size_t q : wins) reversible = reversible && !p->steps[q].win.vw_even;
  for (const TileGroup &tg : p->groups)  // the reverse pass sums at most kMaxGroupWindows windows
    reversible = reversible && tg.ta.nwin <= kMaxGroupWindows;
  // the reversing sweep walks the grouped plan: a tile group runs on every
  // set in one launch, forward and backward.  Partials of window q, set b sit
  // in row (q * batch + b) of nblk_row blocks (at least every launch's grid).
  unsigned nblk_row = nblk;
  if (reversible)
    for (const TileGroup &tg : p->groups) nblk_row = std::max(nblk_row, tile_grid(tg.ta));
  // device memory: psi, lam, checkpoints, stash, partials, coefs, cols, scales
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };  // keep every region 256-byte aligned
  const size_t vec = up(batch * stride * sizeof(float2));
  // the grouped plan checkpoints at the first unit start after every cs
  // windows, so each interval but the last holds at least cs windows
  const size_t nckpt_cap = reversible ? nseg + 1 : nseg;
  const size_t off_lam = vec, off_ckpt = 2 * vec, off_stash = off_ckpt + nckpt_cap * vec;
  const size_t off_part = off_stash + (reversible ? 0 : size_t(cs)) * vec;
  const size_t npart = std::max<size_t>(nwin * batch * nblk_row, batch * lblk);
  const size_t nm = std::max<size_t>(p->n_meas, 1);
  const size_t off_coef = off_part + up(npart * sizeof(double));
  const size_t off_cols = off_coef + up(nm * batch * sizeof(float2));
  const size_t off_scale = off_cols + up((std::max<size_t>(nwin, 1) + 1) * sizeof(int));
  const size_t total = off_scale + up((std::max<size_t>(nwin, 1) + 1) * sizeof(double));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (p->adj_cap < total) {
    if (p->adj_mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p->adj_mem);
    }
    p->adj_mem = nullptr;
    p->adj_cap = 0;
    e = hipMalloc(&p->adj_mem, total);
    if (e != hipSuccess) return fail(p->ctx, OWQS_E_NOMEM, "adjoint buffers");
    p->adj_cap = total;
  } else {
    e = hipStreamSynchronize(s);  // the host tables below are reused
    if (e != hipSuccess) return hip_fail(p->ctx, e, "adjoint");
  }
  char *base = static_cast<char *>(p->adj_mem);
  float2 *psi = reinterpret_cast<float2 *>(base);
  float2 *lam = reinterpret_cast<float2 *>(base + off_lam);
  auto ckpt = [&](size_t j) { return reinterpret_cast<float2 *>(base + off_ckpt + j * vec); };
  auto stash = [&](size_t j) { return reinterpret_cast<float2 *>(base + off_stash + j * vec); };
  double *part = reinterpret_cast<double *>(base + off_part);
  float2 *coefs = reinterpret_cast<float2 *>(base + off_coef);  // [m_index * batch + set]
  int *cols = reinterpret_cast<int *>(base + off_cols);
  double *scales = reinterpret_cast<double *>(base + off_scale);
  // per-set window coefficients c = (-1)^o e^{-i theta}, theta = (-1)^s alpha + t pi (Eq. 2)
  p->adj_coefs.assign(nm * batch, make_float2(0.f, 0.f));
  p->adj_cols.assign(std::max<size_t>(nwin, 1) + 1, 0);
  p->adj_scale.assign(std::max<size_t>(nwin, 1) + 1, 1.0);
  std::vector<double> dth(nm, 1.0);  // dtheta/dalpha of each window's measurement
  for (size_t q = 0; q < nwin; ++q) {
    const Step &x = p->steps[wins[q]];
    for (size_t b = 0; b < batch; ++b) {
      const double a = alpha[b * p->n_meas + x.m_index];
      const double th = (x.sig_s ? -a : a) + (x.sig_t ? M_PI : 0.0);
      double cr = std::cos(th), ci = -std::sin(th);
      if (x.outcome) { cr = -cr; ci = -ci; }
      p->adj_coefs[size_t(x.m_index) * batch + b] = make_float2((float)cr, (float)ci);
    }
    dth[x.m_index] = x.sig_s ? -1.0 : 1.0;
    p->adj_cols[q] = x.m_index;
  }
  if (reversible) {  // partial rows follow the grouped plan's window order (a pass may take later windows first)
    size_t q = 0;
    for (const Step &x : p->xsteps) {
      if (x.kind == S_F) {
        const TileGroup &tg = p->groups[x.group];
        for (int w = 0; w < tg.ta.nwin && q < nwin; ++w) p->adj_cols[q++] = p->fuse_m[tg.m_off + w];
      } else if (x.kind == S_J && q < nwin) {
        p->adj_cols[q++] = x.m_index;
      }
    }
    if (q != nwin) return fail(p->ctx, OWQS_E_STATE, "internal error: the grouped plan lost a window");
  }
  for (size_t q = 0; q < nwin; ++q) p->adj_scale[q] = dth[p->adj_cols[q]];
  e = hipMemcpyAsync(coefs, p->adj_coefs.data(), p->adj_coefs.size() * sizeof(float2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cols, p->adj_cols.data(), p->adj_cols.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(scales, p->adj_scale.data(), p->adj_scale.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(grad, 0, batch * std::max(p->n_meas, 1) * sizeof(double), s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "adjoint tables");
  auto dev_step = [](const Step &x) {
    DevStep d{};
    d.kind = (uint8_t)x.kind;
    d.n = (uint8_t)x.n;
    d.b0 = (uint8_t)x.b0;
    d.b1 = (uint8_t)x.b1;
    d.m_index = x.m_index;
    d.host_factor = (float)x.host_factor;
    d.pp = (x.win.swap ? 1u : 0u) | (x.win.neg0 ? 2u : 0u) | (x.win.neg1 ? 4u : 0u) | (x.win.vw_even ? 8u : 0u);
    d.mask_b = x.win.mask_b;
    d.mask_o1 = x.win.mask_o1;
    return d;
  };
  std::vector<DevStep> d(ns);
  for (size_t i = 0; i < ns; ++i) d[i] = dev_step(p->steps[i]);
  std::vector<size_t> win_of(ns, SIZE_MAX);
  for (size_t q = 0; q < nwin; ++q) win_of[wins[q]] = q;
  const int nsets = (int)batch;
  const size_t seg_bytes = vec;
  std::vector<int> obs_bits(nobs);
  for (int32_t k = 0; k < nobs; ++k) obs_bits[k] = p->final_where[obs[k]];
  auto loss_and_seed = [&]() {
    // loss and the adjoint seed lambda = ff^2 W psi; the loss reduction reads
    // `part` before the window partials overwrite it (same stream), and
    // cols[nwin] = 0, scales[nwin] = 1 were uploaded above
    hipError_t r = launch_b_loss(psi, lam, stride, nsets, (int)p->outputs.size(), obs_bits.data(), nobs,
                                 p->final_factor * p->final_factor, part, s);
    if (r == hipSuccess) r = launch_b_reduce(part, 1, nsets, (int)lblk, cols + nwin, scales + nwin, loss, 1, s);
    return r;
  };
  e = launch_b_init(psi, stride, nsets, (int)p->inputs.size(), static_cast<const float2 *>(input_c64), s);
  if (reversible) {
    owqs_status us = upload_fuse(p);
    if (us != OWQS_OK) return us;
    const std::vector<Step> &xs = p->xsteps;
    const size_t nx = xs.size();
    // units of the grouped plan: windows they hold, first window index
    std::vector<size_t> unit_wins(nx, 0), unit_q(nx, 0);
    for (size_t u = 0, q = 0; u < nx; ++u) {
      unit_q[u] = q;
      unit_wins[u] = xs[u].kind == S_F ? size_t(p->groups[xs[u].group].ta.nwin) : xs[u].kind == S_J ? 1 : 0;
      q += unit_wins[u];
    }
    // forward, with a checkpoint at the start of a unit once cs more windows
    // have gone by (the first at the first unit that holds a window)
    std::vector<size_t> seg_start;
    size_t done = 0, next = 0;
    for (size_t u = 0; u < nx && e == hipSuccess; ++u) {
      const Step &x = xs[u];
      if (unit_wins[u] && done >= next) {
        if (seg_start.size() == nckpt_cap) { e = hipErrorInvalidValue; break; }  // cannot happen (see nckpt_cap)
        e = hipMemcpyAsync(ckpt(seg_start.size()), psi, seg_bytes, hipMemcpyDeviceToDevice, s);
        seg_start.push_back(u);
        next = done + size_t(cs);
      }
      if (e != hipSuccess) break;
      if (x.kind == S_F) {
        const TileGroup &tg = p->groups[x.group];
        e = launch_tile_sets(psi, tg.ta, p->dev_fuse + tg.op_off, nsets, stride, coefs, s);
      } else {
        e = launch_b_step(dev_step(x), psi, stride, nsets,
                          x.kind == S_J ? coefs + size_t(x.m_index) * batch : nullptr, s);
      }
      done += unit_wins[u];
    }
    if (e == hipSuccess) e = loss_and_seed();
    // rows of blocks a launch does not fill must read as zero
    if (e == hipSuccess && nwin) e = hipMemsetAsync(part, 0, nwin * batch * nblk_row * sizeof(double), s);
    // backward, one segment at a time from its end state (the next segment's
    // checkpoint, or the final state): each window recovers its input and
    // moves lambda back in the same pass; E, X and Z are their own inverses
    // and adjoints, applied to psi and lambda together (lam is the buffer
    // after psi, so the two are 2 * batch sets of one array when vec holds
    // exactly batch vectors)
    const bool joint = vec == batch * stride * sizeof(float2) && 2 * batch <= 65535;
    for (size_t j = seg_start.size(); j-- > 0 && e == hipSuccess;) {
      const size_t first = seg_start[j], last = j + 1 < seg_start.size() ? seg_start[j + 1] : nx;
      if (j + 1 < seg_start.size()) e = hipMemcpyAsync(psi, ckpt(j + 1), seg_bytes, hipMemcpyDeviceToDevice, s);
      for (size_t u = last; u-- > first && e == hipSuccess;) {
        const Step &x = xs[u];
        if (x.kind == S_F) {
          const TileGroup &tg = p->groups[x.group];
          e = launch_tile_rev(psi, lam, tg.ta, p->dev_fuse + tg.op_off, nsets, stride, coefs, part, (int)unit_q[u],
                              nblk_row, s);
        } else if (x.kind == S_J) {
          e = launch_b_window_rev(dev_step(x), psi, lam, stride, nsets, coefs + size_t(x.m_index) * batch,
                                  part + unit_q[u] * batch * nblk_row, nblk_row, s);
        } else if (joint) {
          e = launch_b_step(dev_step(x), psi, stride, 2 * nsets, nullptr, s);
        } else {
          e = launch_b_step(dev_step(x), psi, stride, nsets, nullptr, s);
          if (e == hipSuccess) e = launch_b_step(dev_step(x), lam, stride, nsets, nullptr, s);
        }
      }
    }
  } else {
    // forward: prefix, then the windowed part with a checkpoint at each segment start
    for (size_t i = 0; i < ns && e == hipSuccess; ++i) {
      const size_t q = win_of[i];
      if (q != SIZE_MAX && q % cs == 0) e = hipMemcpyAsync(ckpt(q / cs), psi, seg_bytes, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = launch_b_step(d[i], psi, stride, nsets, q != SIZE_MAX ? coefs + size_t(d[i].m_index) * batch : nullptr, s);
    }
    if (e == hipSuccess) e = loss_and_seed();
    // backward, one segment at a time: restore, recompute with a stash of the
    // window inputs, then sweep lambda back through the segment
    for (size_t j = nseg; j-- > 0 && e == hipSuccess;) {
      const size_t first = wins[j * cs];
      const size_t last = (j + 1) * cs < nwin ? wins[(j + 1) * cs] : ns;
      e = hipMemcpyAsync(psi, ckpt(j), seg_bytes, hipMemcpyDeviceToDevice, s);
      for (size_t i = first; i < last && e == hipSuccess; ++i) {
        const size_t q = win_of[i];
        if (q != SIZE_MAX) e = hipMemcpyAsync(stash(q - j * cs), psi, seg_bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          e = launch_b_step(d[i], psi, stride, nsets, q != SIZE_MAX ? coefs + size_t(d[i].m_index) * batch : nullptr,
                            s);
      }
      for (size_t i = last; i-- > first && e == hipSuccess;) {
        const size_t q = win_of[i];
        if (q != SIZE_MAX)
          e = launch_b_window_adj(d[i], stash(q - j * cs), lam, stride, nsets, coefs + size_t(d[i].m_index) * batch,
                                  part + q * batch * nblk, s);
        else
          e = launch_b_step(d[i], lam, stride, nsets, nullptr, s);  // E, X, Z are self-adjoint
      }
    }
  }
  if (e == hipSuccess && nwin)
    e = launch_b_reduce(part, (int)nwin, nsets, (int)(reversible ? nblk_row : nblk), cols, scales, grad,
                        (size_t)p->n_meas, s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "adjoint");
  return OWQS_OK;
}


}  // extern "C"
