// Two-site effective-Hamiltonian product: plan ("Tables") and execution.
#pragma once
#include "ctx.h"

namespace bsd {

struct PsiBlk {
  int l, c, r;          // left index, local state of the two sites, right index
  int rows, cols;
  int64_t off;          // element offset
  int row_in_stack;     // row offset inside the right sector's stack
  int prow_in_stack;    // the same in the stack padded to multiples of 8 rows
};

// psi is stored grouped by right sector: for each right sector r, the blocks
// (l, c) with q_l + q_c + q_r = target follow each other (l ascending, then c),
// so they form one tall matrix of stack_rows[r] x d_R(r).
struct PsiLayout {
  std::vector<PsiBlk> blocks;
  std::map<std::tuple<int, int, int>, int> index;
  std::vector<int64_t> stack_off;
  std::vector<int> stack_rows;
  std::vector<int> stack_prows;   // padded stack rows (multiple of 8)
  int64_t n_elems = 0;
};

struct Operand2 {
  bool ok = false, trans = false, ident = false;
  const double* p = nullptr;
  int64_t ld = 0;
  int out = -1;
};

struct GraphEntry {
  const double* psi;
  double* out;
  int precision;
  hipGraphExec_t exec;
};

// streamed right operators: one block of the pack (gathered at prepare time)
struct StreamGather {
  const double* src;
  int64_t off, n;   // destination element offset, elements (rows x ld)
};
struct StreamChunk {
  int64_t elems = 0, pelems = 0;   // float64 pack elements, bf16 plane elements
  size_t host_off = 0;             // byte offset of the pack in pinned host memory
  std::map<std::pair<const double*, bool>, std::pair<int64_t, int64_t>> where;   // build only
  std::vector<StreamGather> gather;                                              // build only
  std::vector<SplitTask> split;    // planes of the pack (split precision)
  DevBuf split_dev;
};

struct HpsiPlan {
  int site = 0, precision = 0;
  std::vector<GraphEntry> graphs;   // captured products, replayed per call
  DevBuf stage_in, stage_out;       // fixed operands of the graph used by Davidson
  ~HpsiPlan();
  PsiLayout lay;
  DevBuf agg, V;
  size_t agg_bytes = 0, v_bytes = 0;
  std::vector<std::unique_ptr<GemmPlan>> phase1, phase2;      // float64 tile lists
  // split precision: psi is cut into bf16 planes, phase 1 multiplies them with
  // the planes of the right operators and stores V^T as planes, phase 2 reads
  // those and the planes of the left operators (arena addressed through tag 3)
  std::vector<std::unique_ptr<GemmPlan>> phase1s, phase2s;
  // split precision: the channels with the largest operators stay float64
  std::vector<std::unique_ptr<GemmPlan>> phase1h, phase2h;
  DevBuf planes, kmaps, split_tasks;
  size_t plane_bytes = 0;
  int n_split_psi = 0;                   // split tasks for psi (run first in every product)
  // phase-2 problem lists per chunk (float64 and plane operands) and the build
  // options of their current tile lists; the autotuner rebuilds from these
  std::vector<std::vector<GemmProblem>> p1_probs, p2_probs, p2s_probs, p2h_probs;
  GemmBuildOpts opts64, opts_planes;
  std::unique_ptr<GemmPlan> diag_plan;   // diagonal of H_eff (rank-1 sector products)
  DevBuf ones, diag, dav_work;
  bool diag_ready = false;
  double useful_flops = 0.0;
  int64_t op_elems = 0;   // elements of the distinct operator blocks one product reads
  // streamed right operators (the environment exceeds the device budget): the
  // right operator blocks of chunk k are copied from pinned host memory into
  // device slot k % 2 on a side stream while chunk k - 1 computes
  bool stream_r = false;
  double stream_delay_ms = 0.0;   // test hook: host sleep before every chunk copy
  std::vector<StreamChunk> schunks;
  void* pack_host = nullptr;
  size_t pack_bytes = 0, slot_bytes = 0, pslot_bytes = 0;
  DevBuf slots, pslots;
  hipStream_t side = nullptr;
  hipEvent_t ev_loaded[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
  size_t nseg = 0;
  int nchannels = 0, naggs = 0;
};

void build_psi_layout(const Block& Lb, const Block& Rb, const SiteSet& C, const Q& target, PsiLayout& lay);
std::unique_ptr<HpsiPlan> build_hpsi_plan(Ctx& ctx, int site, int precision, size_t ws_budget, hipStream_t s,
                                          bool stream_r = false);
void prepare_stream_slots(HpsiPlan& plan, std::vector<std::vector<GemmProblem>>& p1,
                          std::vector<std::vector<GemmProblem>>& p1s, std::vector<std::vector<GemmProblem>>& p1h,
                          hipStream_t s);
// the streamed product, enqueued directly (copies on the plan's side stream);
// delay_ms > 0 holds every copy back by a host sleep (test hook)
void run_hpsi_stream(HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision,
                     double delay_ms = 0.0);
// precision: 0 float64, 1 split-bf16 x3, 2 split-bf16 x6 (the plan is shared)
void run_hpsi(const HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision = 0);
// the same product replayed from a captured hipGraph (captured on first use for
// this (psi, out, precision); kernels only, no memset nodes)
void run_hpsi_graph(HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision = 0);
int profile_hpsi(const HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision, int cap,
                 double* ms, double* flops, double* bytes, int* kind);
void zero_fill(double* p, int64_t n, hipStream_t s);
// rebuild the phase-2 tile lists of every chunk with new schedule options
// which: bit 0 rebuilds the float64 lists, bit 1 the split-bf16 lists
void rebuild_phase2(HpsiPlan& plan, const GemmBuildOpts& o64, const GemmBuildOpts& oplanes, int which = 3);
// time candidate schedules of phase 2 for `precision` on a scratch vector,
// keep the fastest; returns its product time in milliseconds
struct TuneResult {
  double best_ms = 0.0, default_ms = 0.0;
  int n_candidates = 0, best = 0;
};
TuneResult autotune_hpsi(HpsiPlan& plan, int precision, hipStream_t s);
// diagonal of H_eff into the plan's own buffer (computed once per plan)
const double* hpsi_diagonal(HpsiPlan& plan, hipStream_t s);

}  // namespace bsd
