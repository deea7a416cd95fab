/*
 * owqs_oracle.c -- plain, slow, complex128 reference for executing a
 * one-way quantum computer (1WQC) measurement pattern.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library and must never sit on its execution path.
 *
 * What it computes (Sec. 2.2, Sec. 4.1-4.4 of the paper):
 *   - one live state vector psi of 2^n complex128 amplitudes; slot[k] is the
 *     qubit held by index bit k (qubit v <-> bit weight 2^(v-1) in Fig. 5/6);
 *   - N_v   : psi <- psi (x) |+>, the new qubit taking the top bit
 *             (the tensor product with a one-qubit sub-state, Sec. 4.4.1,
 *             Fig. 8(a)->(b));
 *   - E_uv  : negate every amplitude whose u and v bits are both 1
 *             (Sec. 4.4.1, Fig. 5);
 *   - X_v^s / Z_v^s : swap the pairs differing in bit v / negate where bit v
 *             is 1, when the XOR of the outcomes of s is 1 (Sec. 4.4.1);
 *   - M_v^alpha with domains s, t: the angle becomes
 *             theta = (-1)^s alpha + t pi (Eq. 2); the forced outcome o picks
 *             the elimination operator of Eq. 11 (o = 0) or Eq. 12 (o = 1):
 *             new[k] = (psi[k0] + (-1)^o e^{-i theta} psi[k1]) / sqrt(2),
 *             k0/k1 = k with a 0/1 inserted at the measured bit (the j map of
 *             the Fig. 6 second loop, worked in Eq. 21); the outcome
 *             probability is p = sum |new|^2 (Eq. 13); the vector then halves
 *             (qubit elimination, Sec. 4.2) and higher bits move down.
 *             OWQS mode renormalises by 1/sqrt(p) (Eq. 7).  EOWQS mode
 *             (Sec. 4.5) assumes p = 1/2, scales by sqrt(2), and reports an
 *             error when |p/|psi|^2 - 1/2| exceeds 1e-9.
 *   - the patterns' well-formedness rules D0-D3 (Sec. 2.2) are checked.
 *
 * Readings where the paper is garbled or inconsistent:
 *   - measurement basis sign: Eqs. 9-13 and the Fig. 6 code use
 *     coefficient e^{-i alpha} on the |1> component of the elimination
 *     operator; this oracle follows Eqs. 11-12 (Eq. 1 prints the opposite
 *     sign in the ket).
 *   - the Fig. 6 probability loop is garbled; p is taken as the squared norm
 *     of the forced branch (Eq. 13), which is the same number.
 *   - loops bounds printed as "to size/4" are read as exclusive.
 *
 * Error codes: 0 ok, -1 bad argument, -2 pattern violates D0-D3,
 * -3 forced outcome has probability < 1e-12, -4 width over the limit,
 * -5 out of memory, -7 EOWQS mode on a measurement with p != 1/2.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OP_N = 0, OP_E = 1, OP_M = 2, OP_X = 3, OP_Z = 4 };
enum { Q_UNPREPARED = 0, Q_LIVE = 1, Q_MEASURED = 2 };

#define ORACLE_MAX_WIDTH 30

typedef double complex cplx;

/* XOR of the forced outcomes of the qubits in dom[off .. off+len). Returns -1
 * when one of them has not been measured yet (rule D0). */
static int signal_of(const int *dom, int off, int len, const int *state,
                     const int *outcome, int nq) {
  int s = 0;
  for (int k = 0; k < len; ++k) {
    int j = dom[off + k];
    if (j < 0 || j >= nq || state[j] != Q_MEASURED) return -1;
    s ^= outcome[j];
  }
  return s;
}

int owqs_oracle_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/*
 * Run commands [0, stop) of the pattern (stop < 0: all, then gather outputs).
 *
 * Commands are parallel arrays: op, q0, q1 (E's second qubit), alpha (M),
 * s_off/s_len, t_off/t_len index into dom[] (t used by M only).
 * inputs[k] is bit k of the input vector (in_re/in_im, 2^nin entries).
 * outcomes[m] is the forced outcome of the m-th M command; with uniforms
 * non-NULL the outcomes are drawn instead (Fig. 6: outcome 0 when
 * uniforms[m] <= p_0, the probability of the outcome-0 branch, Eq. 13 with
 * the operator of Eq. 11) and written to outcomes[m].
 * On a full run out_re/out_im receive 2^nout amplitudes with outputs[k] at
 * bit k; on a partial run they receive the live vector (2^n_live entries) and
 * live_slots[k] the qubit held by bit k.  probs[m] receives p of the m-th M.
 */
int owqs_oracle_run(int ncmd, const int *op, const int *q0, const int *q1,
                    const double *alpha, const int *s_off, const int *s_len,
                    const int *t_off, const int *t_len, const int *dom,
                    int nin, const int *inputs, int nout, const int *outputs,
                    const double *in_re, const double *in_im,
                    unsigned char *outcomes, const double *uniforms, int mode, int stop,
                    double *out_re, double *out_im, double *probs,
                    int *live_slots, int *n_live_out, int *err_cmd) {
  if (ncmd < 0 || nin < 0 || nout < 0 || nin > ORACLE_MAX_WIDTH) return -1;
  if (err_cmd) *err_cmd = -1;
  /* qubit ids are small non-negative integers */
  int nq = 0;
  for (int k = 0; k < nin; ++k) if (inputs[k] + 1 > nq) nq = inputs[k] + 1;
  for (int k = 0; k < nout; ++k) if (outputs[k] + 1 > nq) nq = outputs[k] + 1;
  for (int c = 0; c < ncmd; ++c) {
    if (q0[c] + 1 > nq) nq = q0[c] + 1;
    if (op[c] == OP_E && q1[c] + 1 > nq) nq = q1[c] + 1;
    if (q0[c] < 0 || (op[c] == OP_E && q1[c] < 0)) return -1;
  }
  int *qstate = calloc((size_t)nq + 1, sizeof(int));
  int *qout = calloc((size_t)nq + 1, sizeof(int));
  int slot[ORACLE_MAX_WIDTH + 1];
  int n = nin;
  int rc = 0;
  if (!qstate || !qout) { free(qstate); free(qout); return -5; }
  for (int k = 0; k < nin; ++k) {
    if (inputs[k] < 0 || qstate[inputs[k]] != Q_UNPREPARED) { rc = -1; goto done_early; }
    qstate[inputs[k]] = Q_LIVE;
    slot[k] = inputs[k];
  }

  size_t cap = (size_t)1 << n;
  cplx *psi = malloc(sizeof(cplx) * cap);
  if (!psi) { rc = -5; goto done_early; }
  for (size_t i = 0; i < cap; ++i) psi[i] = in_re[i] + I * in_im[i];

  int m_index = 0;
  int last = (stop >= 0 && stop < ncmd) ? stop : ncmd;
  int cur = -1;
  for (int c = 0; c < last; ++c) {
    int v = q0[c];
    cur = c;
    if (op[c] == OP_N) {
      /* D2: N only on a fresh non-input qubit */
      if (qstate[v] != Q_UNPREPARED) { rc = -2; goto fail; }
      if (n + 1 > ORACLE_MAX_WIDTH) { rc = -4; goto fail; }
      size_t dim = (size_t)1 << n;
      cplx *grown = malloc(sizeof(cplx) * dim * 2);
      if (!grown) { rc = -5; goto fail; }
      const double r = 1.0 / sqrt(2.0);
      for (size_t i = 0; i < 2 * dim; ++i) grown[i] = psi[i % dim] * r;
      free(psi);
      psi = grown;
      slot[n] = v;
      n += 1;
      qstate[v] = Q_LIVE;
    } else if (op[c] == OP_E) {
      int u = q1[c];
      if (u == v || qstate[v] != Q_LIVE || qstate[u] != Q_LIVE) { rc = -2; goto fail; }
      int bv = -1, bu = -1;
      for (int k = 0; k < n; ++k) { if (slot[k] == v) bv = k; if (slot[k] == u) bu = k; }
      size_t dim = (size_t)1 << n;
      size_t mask = ((size_t)1 << bv) | ((size_t)1 << bu);
#pragma omp parallel for schedule(static)
      for (size_t i = 0; i < dim; ++i)
        if ((i & mask) == mask) psi[i] = -psi[i];
    } else if (op[c] == OP_X || op[c] == OP_Z) {
      if (qstate[v] != Q_LIVE) { rc = -2; goto fail; }
      int s = signal_of(dom, s_off[c], s_len[c], qstate, qout, nq);
      if (s < 0) { rc = -2; goto fail; }
      if (s == 1) {
        int b = -1;
        for (int k = 0; k < n; ++k) if (slot[k] == v) b = k;
        size_t dim = (size_t)1 << n, bit = (size_t)1 << b;
        if (op[c] == OP_X) {
#pragma omp parallel for schedule(static)
          for (size_t i = 0; i < dim; ++i) {
            if ((i & bit) == 0) {
              cplx t = psi[i];
              psi[i] = psi[i | bit];
              psi[i | bit] = t;
            }
          }
        } else {
#pragma omp parallel for schedule(static)
          for (size_t i = 0; i < dim; ++i)
            if (i & bit) psi[i] = -psi[i];
        }
      }
    } else if (op[c] == OP_M) {
      if (qstate[v] != Q_LIVE) { rc = -2; goto fail; }
      for (int k = 0; k < nout; ++k) if (outputs[k] == v) { rc = -2; goto fail; } /* D3 */
      int s = signal_of(dom, s_off[c], s_len[c], qstate, qout, nq);
      int t = signal_of(dom, t_off[c], t_len[c], qstate, qout, nq);
      if (s < 0 || t < 0) { rc = -2; goto fail; }
      double theta = (s ? -alpha[c] : alpha[c]) + (t ? M_PI : 0.0);   /* Eq. 2 */
      cplx coef = cexp(-I * theta);                                   /* Eqs. 11, 12 */
      int b = -1;
      for (int k = 0; k < n; ++k) if (slot[k] == v) b = k;
      size_t half = (size_t)1 << (n - 1);
      size_t low = ((size_t)1 << b) - 1;
      int o;
      if (uniforms) {
        /* probability of outcome 0 relative to the current norm */
        double p0 = 0.0, nrm = 0.0;
        const double r0 = 1.0 / sqrt(2.0);
#pragma omp parallel for schedule(static) reduction(+ : p0, nrm)
        for (size_t k = 0; k < half; ++k) {
          size_t k0 = ((k >> b) << (b + 1)) | (k & low);
          size_t k1 = k0 | ((size_t)1 << b);
          cplx val = (psi[k0] + coef * psi[k1]) * r0;
          p0 += creal(val) * creal(val) + cimag(val) * cimag(val);
          nrm += creal(psi[k0]) * creal(psi[k0]) + cimag(psi[k0]) * cimag(psi[k0]) +
                 creal(psi[k1]) * creal(psi[k1]) + cimag(psi[k1]) * cimag(psi[k1]);
        }
        o = (nrm > 0.0 && uniforms[m_index] <= p0 / nrm) ? 0 : 1;
        outcomes[m_index] = (unsigned char)o;
      } else {
        o = outcomes[m_index] & 1;
      }
      if (o) coef = -coef;
      cplx *next = malloc(sizeof(cplx) * (half ? half : 1));
      if (!next) { rc = -5; goto fail; }
      const double r = 1.0 / sqrt(2.0);
      double p = 0.0, norm_before = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : p, norm_before)
      for (size_t k = 0; k < half; ++k) {
        size_t k0 = ((k >> b) << (b + 1)) | (k & low);
        size_t k1 = k0 | ((size_t)1 << b);
        cplx val = (psi[k0] + coef * psi[k1]) * r;
        next[k] = val;
        p += creal(val) * creal(val) + cimag(val) * cimag(val);
        norm_before += creal(psi[k0]) * creal(psi[k0]) + cimag(psi[k0]) * cimag(psi[k0]) +
                       creal(psi[k1]) * creal(psi[k1]) + cimag(psi[k1]) * cimag(psi[k1]);
      }
      if (probs) probs[m_index] = p;
      if (p < 1e-12) { free(next); rc = -3; goto fail; }
      double scale;
      if (mode == 1) {
        if (fabs(p / norm_before - 0.5) > 1e-9) { free(next); rc = -7; goto fail; }
        scale = sqrt(2.0);
      } else {
        scale = 1.0 / sqrt(p);
      }
      for (size_t k = 0; k < half; ++k) next[k] *= scale;
      free(psi);
      psi = next;
      for (int k = b; k < n - 1; ++k) slot[k] = slot[k + 1];
      n -= 1;
      qstate[v] = Q_MEASURED;
      qout[v] = o;
      m_index += 1;
    } else {
      rc = -1;
      goto fail;
    }
  }

  if (stop >= 0 && stop < ncmd) {
    size_t dim = (size_t)1 << n;
    for (size_t i = 0; i < dim; ++i) { out_re[i] = creal(psi[i]); out_im[i] = cimag(psi[i]); }
    for (int k = 0; k < n; ++k) live_slots[k] = slot[k];
    *n_live_out = n;
    free(psi);
    goto done_early;
  }

  /* D3: exactly the outputs are still live */
  if (n != nout) { rc = -2; goto fail_end; }
  int where[ORACLE_MAX_WIDTH];
  for (int k = 0; k < nout; ++k) {
    where[k] = -1;
    for (int j = 0; j < n; ++j) if (slot[j] == outputs[k]) where[k] = j;
    if (where[k] < 0) { rc = -2; goto fail_end; }
  }
  {
    size_t dim = (size_t)1 << n;
    for (size_t x = 0; x < dim; ++x) {
      size_t live = 0;
      for (int k = 0; k < nout; ++k) if ((x >> k) & 1) live |= (size_t)1 << where[k];
      out_re[x] = creal(psi[live]);
      out_im[x] = cimag(psi[live]);
    }
  }
  if (n_live_out) *n_live_out = n;
  free(psi);
  goto done_early;

fail:
  if (err_cmd) *err_cmd = cur;
fail_end:
  free(psi);
done_early:
  free(qstate);
  free(qout);
  return rc;
}
