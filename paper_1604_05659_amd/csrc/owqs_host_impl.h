// owqs_host_impl.h -- the pattern and context objects of libowqs and the
// host functions shared by its source files (owqs_host.cpp: loading, plans,
// runs and read-out; owqs_substate_host.cpp: the sub-state executor;
// owqs_sample_host.cpp: drawn outcomes; owqs_adjoint_host.cpp: the adjoint
// sweep).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/owqs.h"
#include "owqs_pattern_access.h"
#include "owqs_internal.h"

struct owqs_ctx {
  int device = 0;
  std::string last_error;
  // batched runs (owqs_run_batch): the last batch captured as one graph, with
  // the device tables its kernels read, replayed while the call's arguments
  // and the patterns' plans stay the same
  struct Batch {
    std::vector<uint64_t> key;      // what the graph was built for
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *dev = nullptr;            // device tables (items, start/read rows, tile and finish entries)
    size_t dev_cap = 0;
    hipStream_t cap = nullptr;      // capture stream
    hipStream_t side[5] = {};       // one branch of the graph per LDS width class (default priority)
    hipEvent_t fork = nullptr;
    hipEvent_t join[5] = {};
    hipEvent_t done = nullptr;      // recorded after every replay
    size_t nodes = 0;               // kernels captured
  } batch;
  // the allocation-free entry point's device array on this device (its
  // address from hipGetSymbolAddress, resolved when the context is created)
  void *noalloc = nullptr;
};

namespace owqs {

enum StepKind : int { S_N = 0, S_E = 1, S_M = 2, S_X = 3, S_Z = 4, S_J = 5, S_F = 7 };

struct Step {
  int kind;
  int n;       // live width before the step
  int b0, b1;  // slots
  float2 coef;
  double host_factor;
  int m_index;
  Window win;
  int sig_s, sig_t, outcome;  // M / window: resolved signals and forced outcome
  int group;                  // S_F: index into the pattern's tile groups
  bool half;                  // S_J in OWQS mode: p = 1/2 is recorded without a reduction (half_prob)
};

struct TileGroup {
  TileArgs ta;
  size_t op_off;  // first FuseOp of the group in the pattern's table
  size_t m_off;   // first window's measurement index in the pattern's m table
  bool half;      // OWQS mode: it has windows, each with an odd E(v, w) count (p = 1/2 exactly), and
                  // runs without a reduction (mark_half)
  bool renorm;    // half, and it ends a run of such windows: its output norm resets sigma (mark_half)
  // the group's commands with runs of windows on one round position composed
  // (DK_U), for passes without window sums and without drawn outcomes:
  // mnops rows from mop_off in the pattern's composed table (0: none)
  size_t mop_off;
  int mnops;
};

// Sub-state executor (OWQS_EXEC_SUBSTATES).  A chain is one sub-state's
// region of the arena, kept by the sub-state that is the base of every merge
// it takes part in.
enum SubKind : int { SS_INIT = 0, SS_N = 1, SS_E = 2, SS_X = 3, SS_Z = 4, SS_M = 5, SS_KRON = 6, SS_J = 7 };

struct SubStep {
  int kind;
  int chain;         // the sub-state acted on
  int n;             // its width before the step
  int b0, b1;        // slots
  int top, top_n;    // SS_KRON: the sub-state merged in, and its width
  float2 coef;       // SS_M, SS_J: (-1)^o e^{-i theta}
  double host_factor;
  int m_index;
  Window win;        // SS_J: the fused window N w; E's; M v; X/Z on w
  bool half;         // SS_J in OWQS mode: p = 1/2 recorded without a reduction
};

// One entry of the sub-state executor's launch order: a plan step, or a tile
// pass over a run of one sub-state's window/E/X/Z steps.
struct SubRun {
  int step;   // index into ss_steps; -1 for a tile pass
  int group;  // index into ss_groups; -1 for a plan step
  int chain;  // the sub-state acted on
};

struct SubChain {
  size_t off = 0;               // first amplitude in the arena
  int maxw = 0;                 // widest it gets (its region holds 2^maxw amplitudes, at least 4)
  std::vector<int> at;          // dense qubit at each slot, at the end of the plan
  double pend = 1.0;            // host factor at the end of the plan
  bool merged = false;          // merged into another chain
};

struct SubFactor {
  int chain;
  std::vector<int> qubits;      // dense, in output order
  std::vector<int> where;       // slot of each, same order
  uint64_t mask = 0;            // output bits held
};

struct Cmd {
  int op;
  int q0, q1;  // dense qubit indices
  double angle;
  std::vector<int> s, t;  // dense qubit indices
};


constexpr size_t kTraceStride = OWQS_MAX_WIDTH + 1;

}  // namespace owqs

using namespace owqs;

struct owqs_pattern {
  owqs_ctx *ctx = nullptr;
  std::vector<Cmd> cmds;
  std::vector<int> inputs, outputs;  // dense
  int nq = 0;
  int n_meas = 0;
  int max_live = 0;
  std::vector<double> angles;     // per M
  std::vector<uint8_t> outcomes;  // per M
  owqs_mode mode = OWQS_MODE_OWQS;
  owqs_exec exec = OWQS_EXEC_AUTO;

  // compiled plan
  bool dirty = true;
  std::vector<Step> steps;
  std::vector<int> final_where;  // slot of outputs[k]
  double final_factor = 1.0;
  int plan_width = 0;            // largest live width the plan reaches

  int tile_bits = 0;  // 0: automatic (max(10, min(12, n - 8))); else 10..13
  // OWQS: windows with p = 1/2 exactly recorded without a sum, at most this
  // many in a row (kHalfRun; 0 after owqs_set_sum_all(p, 1): every M sums)
  int half_cap = kHalfRun;
  // execution steps of the global-memory path: the plan with runs of
  // window/E/X/Z steps grouped into tile passes (S_F)
  std::vector<Step> xsteps;
  std::vector<TileGroup> groups;
  std::vector<FuseOp> fuse_ops;
  std::vector<int> fuse_m;        // measurement index of every window of every group
  std::vector<FuseOp> fuse_mops;  // composed copies of the groups' commands (TileGroup::mop_off)
  // per map of fuse_mops: its row there, its window count, its windows' rows
  // in fuse_ops (drawn runs compose the resolved rows on the device)
  std::vector<int> fuse_msrc;
  FuseOp *dev_fuse = nullptr;     // fuse_ops, then fuse_m (as int), then fuse_mops in one allocation
  size_t dev_fuse_cap = 0;
  bool dev_fuse_valid = false;

  // the plan as a device command table (LDS-resident runs); dev_nsteps rows
  // (fewer than steps when window runs were composed, EOWQS)
  size_t dev_nsteps = 0;
  DevStep *dev_steps = nullptr;
  size_t dev_steps_cap = 0;
  bool dev_steps_valid = false;

  // the plan captured as a HIP graph (kernels only; replayed by owqs_run)
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  // device memory
  float2 *psi = nullptr;
  size_t psi_cap = 0;  // amplitudes
  void *book_mem = nullptr;
  float2 *stage = nullptr;  // device staging for reads into host memory (2^nout)
  DevBook book{};
  // adjoint buffers (owqs_adjoint), grown on demand
  void *adj_mem = nullptr;
  size_t adj_cap = 0;
  std::vector<float2> adj_coefs;   // host copies kept alive for the async uploads
  std::vector<int> adj_cols;
  std::vector<double> adj_scale;

  // lockstep runs (owqs_run_range): the plain plan, one step per non-trivial
  // command, with the state after every command
  bool lk_valid = false;
  std::vector<Step> lk_steps;
  std::vector<size_t> lk_step_end;   // steps emitted by commands 0..i
  std::vector<int> lk_width;         // live width after command i
  std::vector<double> lk_pending;    // host factor of the live vector after command i
  std::vector<int> lk_qubits;        // dense qubit at each bit after command i (stride kTraceStride)
  size_t lk_next = SIZE_MAX;         // first command not yet run by the ranged run in progress
  bool lk_ran = false;

  std::vector<int32_t> user_id;  // dense qubit index -> caller's id

  // drawn outcomes (owqs_set_uniforms): the plain plan with every signal and
  // measurement coefficient resolved on the device
  struct SStep {
    int kind, n, b0, b1, m;
    double alpha, host_factor;
    SigRef s, t;
    Window win;             // S_J: the window's sign masks (its folds are resolved on the device)
    int fold_off, fold_len; // S_J: its corrections in s_folds
    bool half;              // S_J: p = 1/2 recorded without the sum (at most kHalfRun in a row)
  };
  bool sampling = false;
  std::vector<double> uniforms;
  bool s_valid = false;
  std::vector<SStep> s_steps;
  std::vector<int> s_dom;           // measurement indices of the signal domains
  std::vector<FoldRef> s_folds;     // corrections folded into drawn windows
  // every M a window with p = 1/2 and no other correction: the outcomes follow
  // from the uniforms alone, so a run is the fused plan with its window
  // coefficients and folds taken from a per-run device table
  bool s_analytic = false;
  void *a_mem = nullptr;            // coefficients (float2 per M), folds (3 int per M), then the drawn windows
  size_t a_cap = 0;
  bool a_wins_valid = false;        // the drawn-window table in a_mem matches s_steps
  bool fuse_patched = false;        // drawn runs wrote coefficients into dev_fuse: forced runs upload it again
  hipGraph_t a_graph = nullptr;
  hipGraphExec_t a_exec = nullptr;
  bool an_ran = false;
  std::vector<int> s_final_where;
  double s_final_factor = 1.0;
  void *s_mem = nullptr;            // uniforms, outcomes, coefficient, domains
  size_t s_cap = 0;
  bool s_uploaded = false;          // uniforms and domains are on the device
  hipGraph_t s_graph = nullptr;
  hipGraphExec_t s_exec = nullptr;
  bool sampled_ran = false;

  // sub-state executor (OWQS_EXEC_SUBSTATES)
  std::vector<int32_t> ss_in_nq;    // input factorization (qubits per factor, input order); empty: one factor
  std::vector<SubStep> ss_steps;
  std::vector<SubChain> ss_chains;
  std::vector<SubFactor> ss_factors;
  std::vector<int> ss_vanished;     // chains whose qubits were all measured (a scalar each)
  std::vector<SubRun> ss_run;       // launch order (tile passes per sub-state)
  std::vector<TileGroup> ss_groups;
  std::vector<FuseOp> ss_fuse_ops;
  std::vector<int> ss_fuse_m;
  std::vector<FuseOp> ss_fuse_mops; // composed copies of the sub-state groups' commands (TileGroup::mop_off)
  FuseOp *ss_dev_fuse = nullptr;    // ss_fuse_ops, then ss_fuse_m (as int), then ss_fuse_mops
  size_t ss_dev_fuse_cap = 0;
  bool ss_dev_fuse_valid = false;
  int ss_width = 0;                 // widest sub-state
  bool ss_plan_ok = true;           // every step fits its sub-state's region
  size_t ss_arena = 0;              // amplitudes
  float2 *ss_mem = nullptr;
  size_t ss_mem_cap = 0;
  double *ss_sigma = nullptr;       // one FP64 scale per chain
  size_t ss_sigma_cap = 0;
  float2 *ss_stage = nullptr;       // read-out: factors, then the scalars
  size_t ss_stage_cap = 0;
  hipGraph_t ss_graph = nullptr;
  hipGraphExec_t ss_exec = nullptr;
  int ss_graph_reduce = -1;
  bool ss_ran = false;

  uint64_t plan_gen = 0;  // process-wide number of the last compile (batched runs key their graph on it)
  bool ran = false;
  bool out_in_order = false;  // the last run left the read-out (ordered, scaled) at psi[0 .. 2^nout)
  bool batch_ran = false;  // the last run was an LDS batch (outputs went straight to the caller)
  int ran_mode = 0;
  int graph_reduce = -1;
};

namespace owqs {

// ---- owqs_host.cpp
owqs_status fail(owqs_ctx *ctx, owqs_status st, const std::string &msg);
owqs_status hip_fail(owqs_ctx *ctx, hipError_t e, const char *what);
int signal(const std::vector<int> &dom, const std::vector<int> &outcome_of);
void compile(owqs_pattern *p);
owqs_status width_guard(owqs_pattern *p);
owqs_status ensure_device(owqs_pattern *p, bool need_psi = true);
void end_ranged(owqs_pattern *p);
owqs_status upload_fuse(owqs_pattern *p);
// Group runs of window/E/X/Z steps into tile passes (S_F steps in `out`),
// looking up to kGroupLookahead steps ahead past at most kGroupSkipMax steps
// left for later passes.
constexpr size_t kGroupLookahead = 2048;
constexpr size_t kGroupSkipMax = 512;
bool commute_steps(const Step &a, const Step &b);
void group_steps(const std::vector<Step> &steps, int mode, int tile_bits, std::vector<Step> &out,
                 std::vector<TileGroup> &groups, std::vector<FuseOp> &fops, std::vector<int> &fm,
                 bool big_half = false, std::vector<FuseOp> *mops = nullptr, std::vector<int> *msrc = nullptr);
// The commands of one group (nops rows) with every run of two or more
// windows in a row on one register-round position composed into one DK_U
// row; false (and `out` unchanged) when nothing composes.
bool merge_round_windows(const FuseOp *ops, int nops, int tile_bits, std::vector<FuseOp> &out,
                         std::vector<int> *src = nullptr);
// Copy a tile-pass command table (FuseOps, then the windows' measurement
// indices as int, then the composed commands `mops` from a FuseOp boundary)
// to the device, growing `dev` as needed.
owqs_status upload_fuse_table(owqs_ctx *ctx, const std::vector<FuseOp> &fops, const std::vector<int> &fm,
                              FuseOp *&dev, size_t &cap, const std::vector<FuseOp> *mops = nullptr);
// Rows before the composed commands in a table upload_fuse_table wrote.
size_t fuse_mops_base(size_t nfops, size_t nfm);
int *fuse_m_dev(owqs_pattern *p);
// An OWQS window with an odd E(v, w) count: p = 1/2 exactly, no reduction.
bool half_prob(const Step &x, int reduce);
// Error feedback for the FP32 rounding of the factors of such windows.
double rounded_factor(double h, double &e);
// Decide which windows and tile groups with p = 1/2 skip their reduction.
void mark_half(std::vector<Step> &xs, std::vector<TileGroup> &groups, int cap);
int reduce_of(const owqs_pattern *p);
struct Profile {
  int64_t *counts;
  double *ms;
  double *bytes;
};
// With ctab / ftab: the windows take their coefficient and folds from these
// per-run device tables (coefficient of M m at ctab[m], folds at ftab[3 m]).
// psi_over / book_over (non-null): run on that live vector and bookkeeping
// instead of the pattern's own (the allocation-free entry point).
// groups_patched: the tile passes take their windows' coefficients and folds
// from their own command rows (written on the device) rather than ctab/ftab.
hipError_t launch_range(owqs_pattern *p, const std::vector<Step> &xs, size_t i0, size_t i1, int reduce,
                        hipStream_t s, std::vector<hipEvent_t> *ev, const float2 *ctab = nullptr,
                        const int *ftab = nullptr, float2 *psi_over = nullptr, const DevBook *book_over = nullptr,
                        bool groups_patched = false);
LdsItem lds_proto(const owqs_pattern *p);
// Address of the allocation-free entry point's device array on `device`
// (resolved once per device with that device current; owqs_noalloc.hip).
hipError_t noalloc_scratch(int device, void **out);

// ---- owqs_substate_host.cpp
void compile_substates(owqs_pattern *p);
void drop_ss_graph(owqs_pattern *p);
bool substates(const owqs_pattern *p);
owqs_status refuse_substates(owqs_pattern *p, const char *what);
// Input factor k (2^nqs[k] complex64) holds the next nqs[k] inputs.
owqs_status run_substates(owqs_pattern *p, const void *const *factors, const int32_t *nqs, size_t nf,
                          int on_device, void *stream, Profile *prof = nullptr);
// Read every factor (scaled, its qubits in output order) and the scalar of
// the vanished sub-states into ss_stage: factor f at offs[f], the scalar at
// offs.back().
owqs_status stage_substates(owqs_pattern *p, hipStream_t s, std::vector<uint64_t> &offs);

// ---- owqs_sample_host.cpp
void compile_sampled(owqs_pattern *p);
owqs_status run_sampled(owqs_pattern *p, const void *input, size_t n_amps, int input_on_device, void *stream);
// Device layout of s_mem: uniforms (double), outcomes (int), coefficient
// (float2) and a window's folds (3 int) in one 256-byte slot, domains (int),
// folded corrections (FoldRef), each 256-byte aligned.
struct SampleMem {
  double *u;
  int *outc;
  float2 *coef;
  int *fold;
  int *dom;
  FoldRef *folds;
};
SampleMem sample_mem(owqs_pattern *p);

}  // namespace owqs
