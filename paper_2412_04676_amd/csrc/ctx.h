// Library context: integrals, MPS site tensors and renormalized blocks.
#pragma once
#include "internal.h"

namespace bsd {

// One MPS site tensor on the device: blocks (q_left, s) of shape
// d_left(q_left) x d_right(q_left + q_s), bond labels, row-major compact.
struct SiteTensor {
  bool set = false;
  Basis left, right;         // bond labels
  struct Blk {
    int l, r, s;             // basis indices and local state
    int rows, cols;
    int64_t off;             // element offset in dev
  };
  std::vector<Blk> blocks;
  std::map<std::pair<int, int>, int> by_ls;   // (left index, s) -> block
  DevBuf mem;
  const double* ptr(int b) const { return static_cast<const double*>(mem.p) + blocks[b].off; }
};

struct HpsiPlan;

struct Ctx {
  int L = 0, na = 0, nb = 0;
  Q target;
  Integrals ints;
  bool have_ints = false;
  std::vector<SiteTensor> sites;
  std::map<int, std::unique_ptr<Block>> left, right;   // keyed by bond
  std::map<std::pair<int, int>, std::shared_ptr<HpsiPlan>> plans;  // (site, precision)
  DevBuf ws;                 // scratch for renormalization
  size_t renorm_ws_budget = (size_t)8 << 30;   // per batch of new operators
  int right_normal_from = 1 << 30;   // right blocks at bonds >= this keep normal operators
  // statistics
  struct Stats {
    double sec[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // wall seconds per phase (Fig. 9 categories)
    double io_exposed_s = 0.0;
    double hpsi_flops = 0.0;
    int64_t hpsi_calls = 0, dav_calls = 0, dav_iters = 0, truncations = 0;
    int64_t bytes_packed = 0, bytes_unpacked = 0, bytes_d2h = 0, bytes_h2d = 0;
  } st;
  std::map<const void*, hipEvent_t> staging_busy;   // last use of each staging buffer
  double side_delay_ms = 0.0;                       // host delay before each side-stream copy
  size_t hpsi_ws_default = (size_t)16 << 30;
  size_t hbm_budget = 0;
  bool heavy_fp64 = true;   // split products keep the largest-operator channels in float64
  size_t stream_chunk_bytes = 0;   // right operators per chunk (0: no cap; 1 GiB when streaming)
  double last_hpsi_flops = 0.0;
  double renorm_flops = 0.0;     // useful flops of the grouped-GEMM phases
  double renorm_wall_s = 0.0;    // wall time of renormalization steps
  double renorm_dev_s = 0.0;     // of it: from each launch to its stream sync
  int64_t renorm_steps = 0;
  ~Ctx();
};

void renormalize_left_block(Ctx& ctx, int bond, hipStream_t s);   // bond -> bond+1
void renormalize_right_block(Ctx& ctx, int bond, hipStream_t s);  // bond -> bond-1
void make_vacuum_blocks(Ctx& ctx);
Block* get_block(Ctx& ctx, bool left, int bond);

}  // namespace bsd
