// C ABI of the library (declared in include/bsdmrg.h).
#include "../../include/bsdmrg.h"

#include <chrono>
#include <cstddef>
#include <cmath>
#include <thread>

#include "davidson.h"
#include "stvec.h"
#include "truncate.h"

struct bsdmrg_ctx {
  bsd::Ctx c;
};

namespace bsd {

static thread_local std::string g_err;
void set_last_error(const std::string& m) { g_err = m; }

static hipStream_t S(bsdmrg_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

static double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A host function on a stream that sleeps: holds back the copies queued
// after it on the side stream (forces the blocking fetch in tests).
static void sleep_host_fn(void* arg) {
  const double ms = *static_cast<double*>(arg);
  delete static_cast<double*>(arg);
  std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(ms * 1000.0)));
}
static void delay_on(hipStream_t s, double ms) {
  BSD_HIP(hipLaunchHostFunc(s, sleep_host_fn, new double(ms)));
}

// adds the wall time of its scope to one phase of the context statistics
struct PhaseTimer {
  double* acc;
  double t0;
  PhaseTimer(Ctx& c, int ph) : acc(&c.st.sec[ph]), t0(wall_now()) {}
  ~PhaseTimer() { *acc += wall_now() - t0; }
};

template <class F>
static int guard(F&& f) {
  try {
    f();
    return BSDMRG_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return BSDMRG_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return BSDMRG_EINVAL;
  }
}

static std::vector<FamilyView> block_views(const Block& b, bool left) {
  std::vector<FamilyView> v;
  uint64_t tag = 0;
  for (const auto& f : b.fams) {
    FamilyView x;
    x.tag = ((uint64_t)(left ? 0 : 1) << 63) | ((uint64_t)b.first << 40) | ((uint64_t)b.last << 20) | tag++;
    x.dq = f.sk.dq;
    x.n_layers = (int)f.keys.size();
    for (const auto& sb : f.sk.blocks) {
      x.bq.push_back(b.basis.q[sb.in]);
      x.rows.push_back(sb.rows);
      x.cols.push_back(sb.cols);
      x.ld.push_back(sb.ld);
      x.off.push_back(sb.off);
    }
    x.layer_stride = f.sk.layer_stride;
    x.data = f.dev;
    v.push_back(std::move(x));
  }
  return v;
}

static std::vector<FamilyView> desc_views(int n, const bsdmrg_family_desc* d) {
  BSD_CHECK(n >= 0 && (n == 0 || d != nullptr), BSDMRG_EINVAL, "bad family list");
  std::vector<FamilyView> v;
  for (int i = 0; i < n; ++i) {
    const auto& f = d[i];
    BSD_CHECK(f.n_layers >= 0 && f.n_blocks >= 0, BSDMRG_EINVAL, "negative family sizes");
    BSD_CHECK(f.n_blocks == 0 || (f.block_q && f.rows && f.cols && f.ld && f.elem_offset), BSDMRG_EINVAL,
              "missing block arrays");
    BSD_CHECK(f.n_layers == 0 || f.n_blocks == 0 || f.data != nullptr, BSDMRG_EINVAL, "missing data pointer");
    BSD_CHECK(((uintptr_t)f.data % 16) == 0, BSDMRG_EINVAL, "family data must be 16-byte aligned");
    FamilyView x;
    x.tag = f.tag;
    x.dq = {f.dq[0], f.dq[1]};
    x.n_layers = f.n_layers;
    int64_t maxend = 0;
    for (int b = 0; b < f.n_blocks; ++b) {
      BSD_CHECK(f.rows[b] >= 0 && f.cols[b] >= 0 && f.ld[b] >= f.cols[b] && f.elem_offset[b] >= 0, BSDMRG_EINVAL,
                "bad block geometry");
      x.bq.push_back({f.block_q[2 * b], f.block_q[2 * b + 1]});
      x.rows.push_back(f.rows[b]);
      x.cols.push_back(f.cols[b]);
      x.ld.push_back(f.ld[b]);
      x.off.push_back(f.elem_offset[b]);
      if (f.rows[b] > 0) maxend = std::max<int64_t>(maxend, f.elem_offset[b] + (int64_t)(f.rows[b] - 1) * f.ld[b] + f.cols[b]);
    }
    BSD_CHECK(f.n_layers <= 1 || f.layer_stride >= maxend, BSDMRG_EINVAL, "layers overlap");
    x.layer_stride = f.layer_stride;
    x.data = f.data;
    v.push_back(std::move(x));
  }
  return v;
}

static Block* need_block(Ctx& c, int side, int bond) {
  BSD_CHECK(side == BSDMRG_LEFT || side == BSDMRG_RIGHT, BSDMRG_EINVAL, "side must be LEFT or RIGHT");
  Block* b = get_block(c, side == BSDMRG_LEFT, bond);
  BSD_CHECK(b != nullptr, BSDMRG_ESTATE, "block not built");
  return b;
}

static void ensure_splan(Block& b, hipStream_t s) {
  if (!b.splan) b.splan = serial_plan(block_views(b, b.left), s, true);
}

// Back a released block with device memory again.  With stable addresses
// (virtual memory management) every pointer into the block stays valid: the
// serializer descriptors and the product plans are kept.  Otherwise the
// families move and everything that points into them is rebuilt.  The unpack
// that follows writes every element, so the memory is not cleared.
static void reacquire_block(Ctx& c, Block& b) {
  b.mem->acquire_physical();
  if (!b.mem->stable()) {
    for (size_t i = 0; i < b.fams.size(); ++i)
      b.fams[i].dev = reinterpret_cast<double*>(static_cast<char*>(b.mem->va) + b.fam_off[i]);
    b.splan.reset();
    c.plans.clear();
  }
  b.resident = true;
}

// Staging buffers shared by offloads and prefetches: the last operation that
// used a buffer records an event (after its D2H copy, or after its unpack), and
// the next operation that writes the buffer waits for it on its own stream.
static void staging_wait(Ctx& c, const void* staging, hipStream_t writer) {
  auto it = c.staging_busy.find(staging);
  if (it != c.staging_busy.end()) BSD_HIP(hipStreamWaitEvent(writer, it->second, 0));
}
static void staging_mark(Ctx& c, const void* staging, hipStream_t last_user) {
  auto it = c.staging_busy.find(staging);
  if (it == c.staging_busy.end()) {
    hipEvent_t e;
    BSD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    it = c.staging_busy.emplace(staging, e).first;
  }
  BSD_HIP(hipEventRecord(it->second, last_user));
}

}  // namespace bsd

using namespace bsd;

extern "C" {

const char* bsdmrg_last_error(void) { return g_err.c_str(); }

int bsdmrg_create(bsdmrg_ctx** out, const bsdmrg_config* cfg) {
  return guard([&] {
    BSD_CHECK(out != nullptr && cfg != nullptr, BSDMRG_EINVAL, "NULL argument");
    const int L = cfg->L, n_alpha = cfg->n_alpha, n_beta = cfg->n_beta;
    BSD_CHECK(L >= 2 && L <= 512, BSDMRG_EINVAL, "L out of range");
    BSD_CHECK(n_alpha >= 0 && n_beta >= 0 && n_alpha <= L && n_beta <= L, BSDMRG_EINVAL,
              "electron counts do not fit");
    BSD_CHECK(cfg->D_max >= 0 && cfg->right_normal_from >= 0, BSDMRG_EINVAL, "negative configuration value");
    BSD_CHECK(cfg->flags == 0, BSDMRG_EINVAL, "unknown configuration flags");
    auto x = std::make_unique<bsdmrg_ctx>();
    x->c.L = L;
    x->c.na = n_alpha;
    x->c.nb = n_beta;
    x->c.target = {n_alpha, n_beta};
    x->c.sites.resize(L);
    if (cfg->hpsi_ws_bytes) x->c.hpsi_ws_default = cfg->hpsi_ws_bytes;
    if (cfg->renorm_ws_bytes) x->c.renorm_ws_budget = cfg->renorm_ws_bytes;
    x->c.hbm_budget = cfg->hbm_budget_bytes;
    if (cfg->right_normal_from) x->c.right_normal_from = cfg->right_normal_from;
    make_vacuum_blocks(x->c);
    *out = x.release();
  });
}

int bsdmrg_destroy(bsdmrg_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    delete ctx;
  });
}

int bsdmrg_load_integrals(bsdmrg_ctx* ctx, const double* h, const double* eri, double e_core) {
  return guard([&] {
    BSD_CHECK(ctx && h && eri, BSDMRG_EINVAL, "NULL argument");
    BSD_CHECK(e_core == 0.0, BSDMRG_EINVAL, "only electronic energies (e_core = 0) are supported");
    const int L = ctx->c.L;
    const size_t n2 = (size_t)L * L, n4 = n2 * n2;
    double mx = 0.0;
    for (size_t i = 0; i < n4; ++i) {
      BSD_CHECK(std::isfinite(eri[i]), BSDMRG_EINVAL, "non-finite integral");
      mx = std::max(mx, std::fabs(eri[i]));
    }
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q) {
        BSD_CHECK(std::isfinite(h[p * L + q]) && std::fabs(h[p * L + q] - h[q * L + p]) <= 1e-12 * (1.0 + std::fabs(h[p * L + q])),
                  BSDMRG_EINVAL, "h is not symmetric");
      }
    const double tol = 1e-12 * std::max(mx, 1e-300);
    auto E = [&](int p, int q, int r, int s) { return eri[(((size_t)p * L + q) * L + r) * L + s]; };
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q)
        for (int r = 0; r < L; ++r)
          for (int s = 0; s < L; ++s) {
            double v = E(p, q, r, s);
            BSD_CHECK(std::fabs(v - E(q, p, r, s)) <= tol && std::fabs(v - E(p, q, s, r)) <= tol &&
                          std::fabs(v - E(r, s, p, q)) <= tol,
                      BSDMRG_EINVAL, "eri violates the 8-fold permutational symmetry");
          }
    ctx->c.ints.L = L;
    ctx->c.ints.h.assign(h, h + n2);
    ctx->c.ints.eri.assign(eri, eri + n4);
    ctx->c.have_ints = true;
    // blocks built from older integrals are stale
    Ctx& c = ctx->c;
    c.plans.clear();
    c.left.clear();
    c.right.clear();
    make_vacuum_blocks(c);
  });
}

static HpsiPlan* get_plan(Ctx& c, int site, int precision, size_t ws, hipStream_t s, bool rebuild);

// A renormalization that builds a block first frees the product plans: the
// new block takes the device memory a plan held (at L=76 D=4096 a plan holds
// tens of GB), and a sweep prepares the next position's plan after it anyway.
// Work queued on the plans' buffers finishes first.
static void release_plans(Ctx& c) {
  if (c.plans.empty()) return;
  BSD_HIP(hipDeviceSynchronize());
  c.plans.clear();
}

// the environment blocks a prepared product reads must be on the device (a
// streamed product reads its right operators from pinned host memory)
static void need_env(Ctx& c, int site, const HpsiPlan* p, Block** Lo = nullptr, Block** Ro = nullptr) {
  Block* Lb = get_block(c, true, site);
  Block* Rb = get_block(c, false, site + 2);
  BSD_CHECK(Lb && Rb, BSDMRG_ESTATE, "environment blocks not built");
  BSD_CHECK(Lb->resident && (Rb->resident || (p && p->stream_r)), BSDMRG_EBUSY, "environment blocks not resident");
  if (Lo) *Lo = Lb;
  if (Ro) *Ro = Rb;
}

static void set_site_tensor_impl(Ctx& c, int site, int n_blocks, const int32_t* meta, const double* data) {
    BSD_CHECK(site >= 0 && site < c.L, BSDMRG_EINVAL, "site out of range");
    BSD_CHECK(n_blocks > 0, BSDMRG_EINVAL, "no blocks");
    SiteTensor T;
    std::map<Q, int> ld, rd;
    int64_t off = 0;
    std::vector<SiteTensor::Blk> blks;
    for (int b = 0; b < n_blocks; ++b) {
      const int32_t* m = meta + 5 * b;
      BSD_CHECK(m[2] >= 0 && m[2] < 4 && m[3] > 0 && m[4] > 0, BSDMRG_EINVAL, "bad block meta");
      Q ql{m[0], m[1]};
      Q qr = ql + kSiteQ[m[2]];
      auto chk = [&](std::map<Q, int>& d, Q q, int v) {
        auto it = d.find(q);
        if (it == d.end()) d[q] = v;
        else BSD_CHECK(it->second == v, BSDMRG_ESHAPE, "inconsistent bond sector dimension");
      };
      chk(ld, ql, m[3]);
      chk(rd, qr, m[4]);
      SiteTensor::Blk x;
      x.s = m[2];
      x.rows = m[3];
      x.cols = m[4];
      x.off = off;
      off += (int64_t)m[3] * m[4];
      blks.push_back(x);
    }
    for (auto& kv : ld) T.left.add(kv.first, kv.second);
    for (auto& kv : rd) T.right.add(kv.first, kv.second);
    for (int b = 0; b < n_blocks; ++b) {
      const int32_t* m = meta + 5 * b;
      Q ql{m[0], m[1]};
      blks[b].l = T.left.find(ql);
      blks[b].r = T.right.find(ql + kSiteQ[m[2]]);
      BSD_CHECK(T.by_ls.find({blks[b].l, blks[b].s}) == T.by_ls.end(), BSDMRG_ESHAPE, "duplicate block");
      T.by_ls[{blks[b].l, blks[b].s}] = b;
    }
    T.blocks = blks;
    T.mem.reserve(std::max<int64_t>(off, 1) * sizeof(double));
    BSD_HIP(hipMemcpy(T.mem.p, data, off * sizeof(double), hipMemcpyHostToDevice));
    T.set = true;
    c.sites[site] = std::move(T);
    // blocks that depend on this site are stale, and so are the products that
    // read them: the product at i reads the left block of bond i (sites < i) and
    // the right block of bond i + 2 (sites >= i + 2)
    for (auto it = c.left.begin(); it != c.left.end();) it = it->first > site ? c.left.erase(it) : std::next(it);
    for (auto it = c.right.begin(); it != c.right.end();) it = it->first <= site ? c.right.erase(it) : std::next(it);
    for (auto it = c.plans.begin(); it != c.plans.end();) {
      const int i = it->first.first;
      it = (i > site || i + 2 <= site) ? c.plans.erase(it) : std::next(it);
    }
}

int bsdmrg_set_site_tensor(bsdmrg_ctx* ctx, int site, int n_blocks, const int32_t* meta, const double* data) {
  return guard([&] {
    BSD_CHECK(ctx && meta && data, BSDMRG_EINVAL, "NULL argument");
    set_site_tensor_impl(ctx->c, site, n_blocks, meta, data);
  });
}

int bsdmrg_get_site_tensor(bsdmrg_ctx* ctx, int site, int* n_blocks, int64_t* n_elems, int32_t* meta,
                           double* data) {
  return guard([&] {
    BSD_CHECK(ctx && n_blocks && n_elems, BSDMRG_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    BSD_CHECK(site >= 0 && site < c.L, BSDMRG_EINVAL, "site out of range");
    const SiteTensor& T = c.sites[site];
    BSD_CHECK(T.set, BSDMRG_ESTATE, "site tensor not set");
    // ascending (q_left, s)
    std::vector<int> order(T.blocks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const Q qx = T.left.q[T.blocks[x].l], qy = T.left.q[T.blocks[y].l];
      if (qx != qy) return qx < qy;
      return T.blocks[x].s < T.blocks[y].s;
    });
    int64_t ne = 0;
    for (const auto& b : T.blocks) ne += (int64_t)b.rows * b.cols;
    *n_blocks = (int)T.blocks.size();
    *n_elems = ne;
    if (!meta) return;
    BSD_CHECK(data != nullptr || ne == 0, BSDMRG_EINVAL, "data is NULL");
    std::vector<double> all(ne);
    if (ne) BSD_HIP(hipMemcpy(all.data(), T.mem.p, ne * sizeof(double), hipMemcpyDeviceToHost));
    int64_t o = 0;
    for (size_t i = 0; i < order.size(); ++i) {
      const auto& b = T.blocks[order[i]];
      const Q ql = T.left.q[b.l];
      int32_t* m = meta + 5 * i;
      m[0] = ql.a;
      m[1] = ql.b;
      m[2] = b.s;
      m[3] = b.rows;
      m[4] = b.cols;
      const int64_t n = (int64_t)b.rows * b.cols;
      std::copy(all.begin() + b.off, all.begin() + b.off + n, data + o);
      o += n;
    }
  });
}

int bsdmrg_truncate(bsdmrg_ctx* ctx, int site, const double* psi, int D, int direction, double* trunc_err,
                    int* D_kept, double* sv, int cap, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && psi && trunc_err && D_kept, BSDMRG_EINVAL, "NULL argument");
    BSD_CHECK(D > 0, BSDMRG_EINVAL, "D must be positive");
    BSD_CHECK(direction == 0 || direction == 1, BSDMRG_EINVAL, "direction must be 0 (left to right) or 1");
    Ctx& c = ctx->c;
    HpsiPlan* p = get_plan(c, site, BSDMRG_FP64, 0, S(stream), false);
    PhaseTimer tm(c, BSDMRG_PH_SVD);
    c.st.truncations += 1;
    TruncResult r = truncate_psi(c, *p, psi, D, direction == 0, p->dav_work, S(stream));
    BSD_CHECK(!r.blocks.empty(), BSDMRG_ESHAPE, "nothing kept");
    std::vector<int32_t> meta;
    std::vector<double> data;
    for (const auto& b : r.blocks) {
      meta.insert(meta.end(), {b.ql.a, b.ql.b, b.s, b.rows, b.cols});
      data.insert(data.end(), b.data.begin(), b.data.end());
    }
    *trunc_err = r.trunc_err;
    *D_kept = r.D_kept;
    if (sv)
      for (int i = 0; i < cap && i < (int)r.sv.size(); ++i) sv[i] = r.sv[i];
    set_site_tensor_impl(c, direction == 0 ? site : site + 1, (int)r.blocks.size(), meta.data(), data.data());
  });
}

int bsdmrg_set_renorm_workspace(bsdmrg_ctx* ctx, size_t bytes) {
  return guard([&] {
    BSD_CHECK(ctx && bytes > 0, BSDMRG_EINVAL, "NULL ctx or zero budget");
    ctx->c.renorm_ws_budget = bytes;
  });
}

int bsdmrg_set_right_normal(bsdmrg_ctx* ctx, int bond) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    BSD_CHECK(bond >= 1, BSDMRG_EINVAL, "bond must be >= 1");
    ctx->c.right_normal_from = std::min(bond, 1 << 30);
  });
}

int bsdmrg_renorm_stats(bsdmrg_ctx* ctx, double* flops, double* wall_s, double* device_s, int64_t* steps) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    const Ctx& c = ctx->c;
    if (flops) *flops = c.renorm_flops;
    if (wall_s) *wall_s = c.renorm_wall_s;
    if (device_s) *device_s = c.renorm_dev_s;
    if (steps) *steps = c.renorm_steps;
  });
}

int bsdmrg_build_env(bsdmrg_ctx* ctx, int side, int bond, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Ctx& c = ctx->c;
    BSD_CHECK(c.have_ints, BSDMRG_ESTATE, "integrals not loaded");
    BSD_CHECK(bond >= 0 && bond <= c.L, BSDMRG_EINVAL, "bond out of range");
    // grow from the nearest block that exists on the way to `bond`
    if (side == BSDMRG_LEFT) {
      int b0 = bond;
      while (b0 > 0 && !get_block(c, true, b0)) --b0;
      PhaseTimer tm(c, BSDMRG_PH_REN_L);
      if (b0 < bond) release_plans(c);
      for (int b = b0; b < bond; ++b) {
        BSD_CHECK(c.sites[b].set, BSDMRG_ESTATE, "site tensor missing");
        Block* cur = get_block(c, true, b);
        BSD_CHECK(cur && cur->resident, BSDMRG_EBUSY, "source block not resident");
        renormalize_left_block(c, b, S(stream));
      }
    } else {
      BSD_CHECK(side == BSDMRG_RIGHT, BSDMRG_EINVAL, "side must be LEFT or RIGHT");
      int b0 = bond;
      while (b0 < c.L && !get_block(c, false, b0)) ++b0;
      PhaseTimer tm(c, BSDMRG_PH_REN_R);
      if (b0 > bond) release_plans(c);
      for (int b = b0; b > bond; --b) {
        BSD_CHECK(c.sites[b - 1].set, BSDMRG_ESTATE, "site tensor missing");
        Block* cur = get_block(c, false, b);
        BSD_CHECK(cur && cur->resident, BSDMRG_EBUSY, "source block not resident");
        renormalize_right_block(c, b, S(stream));
      }
    }
    BSD_HIP(hipStreamSynchronize(S(stream)));
  });
}

int bsdmrg_renormalize(bsdmrg_ctx* ctx, int side, int bond, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Ctx& c = ctx->c;
    BSD_CHECK(c.have_ints, BSDMRG_ESTATE, "integrals not loaded");
    BSD_CHECK(side == BSDMRG_LEFT || side == BSDMRG_RIGHT, BSDMRG_EINVAL, "side must be LEFT or RIGHT");
    const bool left = side == BSDMRG_LEFT;
    BSD_CHECK(left ? (bond >= 0 && bond < c.L) : (bond > 0 && bond <= c.L), BSDMRG_EINVAL, "bond out of range");
    const int site = left ? bond : bond - 1;
    BSD_CHECK(c.sites[site].set, BSDMRG_ESTATE, "site tensor missing");
    Block* cur = get_block(c, left, bond);
    BSD_CHECK(cur != nullptr, BSDMRG_ESTATE, "source block not built");
    BSD_CHECK(cur->resident, BSDMRG_EBUSY, "source block not resident");
    auto& m = left ? c.left : c.right;
    auto it = m.find(left ? bond + 1 : bond - 1);
    if (it != m.end())
      BSD_CHECK(!it->second->offload_pending, BSDMRG_EBUSY, "offload of the target block in flight; wait first");
    PhaseTimer tm(c, left ? BSDMRG_PH_REN_L : BSDMRG_PH_REN_R);
    release_plans(c);
    if (left) renormalize_left_block(c, bond, S(stream));
    else renormalize_right_block(c, bond, S(stream));
    BSD_HIP(hipStreamSynchronize(S(stream)));
  });
}

int bsdmrg_drop_block(bsdmrg_ctx* ctx, int side, int bond) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Ctx& c = ctx->c;
    BSD_CHECK(side == BSDMRG_LEFT || side == BSDMRG_RIGHT, BSDMRG_EINVAL, "side must be LEFT or RIGHT");
    const bool left = side == BSDMRG_LEFT;
    BSD_CHECK(bond > 0 && bond < c.L, BSDMRG_EINVAL, "bond out of range (the vacuum blocks stay)");
    auto& m = left ? c.left : c.right;
    auto it = m.find(bond);
    if (it == m.end()) return;
    BSD_CHECK(!it->second->offload_pending, BSDMRG_EBUSY, "offload in flight; wait first");
    BSD_HIP(hipDeviceSynchronize());
    c.plans.clear();   // plans may reference the block
    m.erase(it);
  });
}

static HpsiPlan* get_plan(Ctx& c, int site, int precision, size_t ws, hipStream_t s, bool rebuild) {
  BSD_CHECK(site >= 0 && site + 1 < c.L, BSDMRG_EINVAL, "site out of range");
  BSD_CHECK(precision >= BSDMRG_FP64 && precision <= BSDMRG_BF16X6, BSDMRG_EINVAL, "unsupported precision");
  auto key = std::make_pair(site, 0);   // one plan serves every precision
  auto it = c.plans.find(key);
  if (it != c.plans.end() && !rebuild) return it->second.get();
  if (ws == 0) ws = c.hpsi_ws_default;
  PhaseTimer tm(c, BSDMRG_PH_TABLES);
  // one product plan at a time: the plans of other positions (a sweep has
  // moved on) and the one being replaced give their device memory back first
  c.plans.clear();
  Block* Lb = get_block(c, true, site);
  Block* Rb = get_block(c, false, site + 2);
  const bool stream = c.hbm_budget > 0 && Lb && Rb && Lb->device_bytes() + Rb->device_bytes() > c.hbm_budget;
  auto p = build_hpsi_plan(c, site, precision, ws, s, stream);
  // a streamed product does not read the right block's memory: the diagonal
  // (which does) is formed now, while the block is resident
  if (stream) hpsi_diagonal(*p, s);
  HpsiPlan* raw = p.get();
  c.plans[key] = std::move(p);
  return raw;
}

int bsdmrg_psi_layout(bsdmrg_ctx* ctx, int site, int* n_blocks, int64_t* n_elems, int32_t* meta, int64_t* offsets) {
  return guard([&] {
    BSD_CHECK(ctx && n_blocks && n_elems, BSDMRG_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    BSD_CHECK(site >= 0 && site + 1 < c.L, BSDMRG_EINVAL, "site out of range");
    Block* Lb = get_block(c, true, site);
    Block* Rb = get_block(c, false, site + 2);
    BSD_CHECK(Lb && Rb, BSDMRG_ESTATE, "environment blocks not built");
    PsiLayout lay;
    SiteSet C = make_siteset(site, 2);
    build_psi_layout(*Lb, *Rb, C, c.target, lay);
    *n_blocks = (int)lay.blocks.size();
    *n_elems = lay.n_elems;
    if (!meta) return;
    BSD_CHECK(offsets != nullptr, BSDMRG_EINVAL, "offsets is NULL");
    for (size_t b = 0; b < lay.blocks.size(); ++b) {
      const PsiBlk& x = lay.blocks[b];
      Q ql = Lb->basis.q[x.l];
      Q qr = c.target - Rb->basis.q[x.r];
      int32_t* m = meta + 8 * b;
      m[0] = ql.a;
      m[1] = ql.b;
      m[2] = x.c / 4;
      m[3] = x.c % 4;
      m[4] = qr.a;
      m[5] = qr.b;
      m[6] = x.rows;
      m[7] = x.cols;
      offsets[b] = x.off;
    }
  });
}

int bsdmrg_hpsi_prepare(bsdmrg_ctx* ctx, int site, int precision, size_t ws_bytes, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    get_plan(ctx->c, site, precision, ws_bytes, S(stream), true);
    BSD_HIP(hipStreamSynchronize(S(stream)));
  });
}

int bsdmrg_hpsi_autotune(bsdmrg_ctx* ctx, int site, int precision, bsdmrg_stream_t stream, double* best_ms,
                         double* default_ms, int* n_candidates) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    HpsiPlan* p = get_plan(ctx->c, site, precision, 0, S(stream), false);
    Block *Lb = nullptr, *Rb = nullptr;
    need_env(ctx->c, site, p, &Lb, &Rb);
    TuneResult r = autotune_hpsi(*p, precision, S(stream));
    if (best_ms) *best_ms = r.best_ms;
    if (default_ms) *default_ms = r.default_ms;
    if (n_candidates) *n_candidates = r.n_candidates;
  });
}

int bsdmrg_hpsi_schedule(bsdmrg_ctx* ctx, int site, int precision, double target_waves, int xcd_order,
                         int wave_max) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    BSD_CHECK(precision >= BSDMRG_FP64 && precision <= BSDMRG_BF16X6, BSDMRG_EINVAL, "unsupported precision");
    BSD_CHECK(target_waves >= 256.0 && target_waves <= 1048576.0, BSDMRG_EINVAL, "target_waves out of [256, 2^20]");
    BSD_CHECK(wave_max >= 16, BSDMRG_EINVAL, "wave_max below 16");
    auto it = ctx->c.plans.find({site, 0});
    BSD_CHECK(it != ctx->c.plans.end(), BSDMRG_ESTATE, "product not prepared");
    HpsiPlan& p = *it->second;
    GemmBuildOpts a = p.opts64, b = p.opts_planes;
    if (precision == BSDMRG_FP64) {
      a.target_waves = target_waves;
      a.xcd_order = xcd_order != 0;
      a.wave_max = wave_max;
    } else {
      b.target_waves = target_waves;
      b.xcd_order = xcd_order != 0;
      b.wave_max = wave_max;
    }
    rebuild_phase2(p, a, b, precision == BSDMRG_FP64 ? 1 : 2);
  });
}

int bsdmrg_hpsi(bsdmrg_ctx* ctx, int site, const double* psi, double* out, int precision, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && psi && out, BSDMRG_EINVAL, "NULL argument");
    BSD_CHECK(psi != out, BSDMRG_EINVAL, "psi and out must not alias");
    HpsiPlan* p = get_plan(ctx->c, site, precision, 0, S(stream), false);
    Block *Lb = nullptr, *Rb = nullptr;
    need_env(ctx->c, site, p, &Lb, &Rb);
    const double* pe = psi + p->lay.n_elems;
    BSD_CHECK(!(out < pe && psi < out + p->lay.n_elems), BSDMRG_EINVAL, "psi and out overlap");
    p->stream_delay_ms = ctx->c.side_delay_ms;
    run_hpsi_graph(*p, psi, out, S(stream), precision);
    Lb->mark_use(S(stream));
    if (Rb->resident) Rb->mark_use(S(stream));
    if (p->stream_r) ctx->c.st.bytes_h2d += (int64_t)p->pack_bytes;
    ctx->c.last_hpsi_flops = p->useful_flops;
    ctx->c.st.hpsi_calls += 1;
    ctx->c.st.hpsi_flops += p->useful_flops;
  });
}

int bsdmrg_hpsi_profile(bsdmrg_ctx* ctx, int site, const double* psi, double* out, int precision,
                        bsdmrg_stream_t stream, int cap, double* ms, double* flops, double* bytes, int* kind,
                        int* n) {
  return guard([&] {
    BSD_CHECK(ctx && psi && out && n && (cap <= 0 || (ms && flops && kind)), BSDMRG_EINVAL, "NULL argument");
    HpsiPlan* p = get_plan(ctx->c, site, precision, 0, S(stream), false);
    Block *Lb = nullptr, *Rb = nullptr;
    need_env(ctx->c, site, p, &Lb, &Rb);
    BSD_CHECK(!p->stream_r, BSDMRG_ESTATE, "per-launch profile of a streamed product is not available");
    *n = profile_hpsi(*p, psi, out, S(stream), precision, cap, ms, flops, bytes, kind);
  });
}

int bsdmrg_davidson(bsdmrg_ctx* ctx, int site, double* psi, const bsdmrg_dav_opts* opts, double* energy,
                    int* iters, double* resid, double* ritz, int cap, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && psi && energy && iters && resid, BSDMRG_EINVAL, "NULL argument");
    HpsiPlan* p = get_plan(ctx->c, site, BSDMRG_FP64, 0, S(stream), false);
    Block *Lb = nullptr, *Rb = nullptr;
    need_env(ctx->c, site, p, &Lb, &Rb);
    DavidsonOpts o;
    if (opts) {
      BSD_CHECK(opts->max_iter > 0 && opts->max_subspace >= 4 && opts->max_subspace <= 30 && opts->restart >= 1 &&
                    opts->restart < opts->max_subspace - 1 && opts->tol > 0 && opts->precond_floor > 0 &&
                    opts->precision >= BSDMRG_FP64 && opts->precision <= BSDMRG_BF16X6 &&
                    (opts->precond == 0 || opts->precond == 1),
                BSDMRG_EINVAL, "bad Davidson options");
      o.precision = opts->precision;
      o.precond = opts->precond;
      o.max_iter = opts->max_iter;
      o.max_sub = opts->max_subspace;
      o.restart = opts->restart;
      o.tol = opts->tol;
      o.precond_floor = opts->precond_floor;
    }
    PhaseTimer tm(ctx->c, BSDMRG_PH_DIAG_H);
    p->stream_delay_ms = ctx->c.side_delay_ms;
    const double* d = hpsi_diagonal(*p, S(stream));
    DavidsonResult r = davidson(*p, d, psi, o, p->dav_work, S(stream));
    ctx->c.st.dav_calls += 1;
    ctx->c.st.dav_iters += r.iters;
    ctx->c.st.hpsi_calls += r.products;
    ctx->c.st.hpsi_flops += r.products * p->useful_flops;
    if (p->stream_r) ctx->c.st.bytes_h2d += (int64_t)p->pack_bytes * r.products;
    *energy = r.energy;
    *iters = r.iters;
    *resid = r.resid;
    if (ritz)
      for (int i = 0; i < cap && i < (int)r.ritz.size(); ++i) ritz[i] = r.ritz[i];
  });
}

int bsdmrg_next_guess(bsdmrg_ctx* ctx, int site, int direction, const double* psi, double* guess,
                      bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && psi && guess, BSDMRG_EINVAL, "NULL argument");
    BSD_CHECK(direction == 0 || direction == 1, BSDMRG_EINVAL, "direction must be 0 (left to right) or 1");
    Ctx& c = ctx->c;
    BSD_CHECK(site >= 0 && site + 1 < c.L, BSDMRG_EINVAL, "site out of range");
    PhaseTimer tm(c, BSDMRG_PH_STVEC);
    next_guess(c, site, direction == 0, psi, guess, c.ws, S(stream));
  });
}

int bsdmrg_hpsi_diagonal(bsdmrg_ctx* ctx, int site, double* diag, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && diag, BSDMRG_EINVAL, "NULL argument");
    HpsiPlan* p = get_plan(ctx->c, site, BSDMRG_FP64, 0, S(stream), false);
    Block *Lb = nullptr, *Rb = nullptr;
    need_env(ctx->c, site, p, &Lb, &Rb);
    const double* d = hpsi_diagonal(*p, S(stream));
    BSD_HIP(hipMemcpyAsync(diag, d, p->lay.n_elems * sizeof(double), hipMemcpyDeviceToDevice, S(stream)));
    Lb->mark_use(S(stream));
    if (Rb->resident) Rb->mark_use(S(stream));
  });
}

int bsdmrg_hpsi_info(bsdmrg_ctx* ctx, int site, int precision, double* flops, int64_t* n_channels,
                     int64_t* n_segments, int64_t* n_aggregates, int64_t* ws_bytes, int64_t* op_elems) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    BSD_CHECK(precision >= BSDMRG_FP64 && precision <= BSDMRG_BF16X6, BSDMRG_EINVAL, "unsupported precision");
    auto it = ctx->c.plans.find({site, 0});
    BSD_CHECK(it != ctx->c.plans.end(), BSDMRG_ESTATE, "product not prepared");
    const HpsiPlan& p = *it->second;
    if (flops) *flops = p.useful_flops;
    if (n_channels) *n_channels = p.nchannels;
    if (n_segments) *n_segments = (int64_t)p.nseg;
    if (n_aggregates) *n_aggregates = p.naggs;
    if (ws_bytes) *ws_bytes = (int64_t)(p.agg_bytes + p.v_bytes + p.plane_bytes);
    if (op_elems) *op_elems = p.op_elems;
  });
}

int bsdmrg_get_block_op(bsdmrg_ctx* ctx, int side, int bond, char kind, int p, int q, int* n_blocks,
                        int64_t* n_elems, int32_t* meta, double* data) {
  return guard([&] {
    BSD_CHECK(ctx && n_blocks && n_elems, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(b->resident, BSDMRG_EBUSY, "block not resident");
    OpKey k;
    k.kind = kind;
    k.p = p;
    k.q = q;
    auto it = b->ops.find(k);
    BSD_CHECK(it != b->ops.end(), BSDMRG_ESTATE, "operator not stored in this block");
    const Family& f = b->fams[it->second.fam];
    int64_t ne = 0;
    for (auto& sb : f.sk.blocks) ne += (int64_t)sb.rows * sb.cols;
    *n_blocks = (int)f.sk.blocks.size();
    *n_elems = ne;
    if (!data) return;
    BSD_CHECK(meta != nullptr, BSDMRG_EINVAL, "meta is NULL");
    std::vector<double> tmp(f.sk.layer_stride);
    BSD_HIP(hipMemcpy(tmp.data(), f.dev + (int64_t)it->second.layer * f.sk.layer_stride,
                      f.sk.layer_stride * sizeof(double), hipMemcpyDeviceToHost));
    int64_t o = 0;
    for (size_t i = 0; i < f.sk.blocks.size(); ++i) {
      const SkBlock& sb = f.sk.blocks[i];
      Q qi = b->basis.q[sb.in], qo = b->basis.q[sb.out];
      int32_t* m = meta + 6 * i;
      m[0] = qi.a;
      m[1] = qi.b;
      m[2] = qo.a;
      m[3] = qo.b;
      m[4] = sb.rows;
      m[5] = sb.cols;
      for (int r = 0; r < sb.rows; ++r)
        for (int cc = 0; cc < sb.cols; ++cc) data[o++] = tmp[sb.off + (int64_t)r * sb.ld + cc];
    }
  });
}

int bsdmrg_block_gemm(int n, const bsdmrg_gemm_desc* probs, int precision, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(n >= 0 && (n == 0 || probs), BSDMRG_EINVAL, "bad problem list");
    BSD_CHECK(precision >= BSDMRG_FP64 && precision <= BSDMRG_BF16X6, BSDMRG_EINVAL, "unsupported precision");
    std::vector<GemmProblem> v;
    for (int i = 0; i < n; ++i) {
      const auto& d = probs[i];
      BSD_CHECK(d.M >= 0 && d.N >= 0 && d.K >= 0, BSDMRG_EINVAL, "negative sizes");
      if (d.M == 0 || d.N == 0) continue;
      BSD_CHECK(d.C && (d.K == 0 || (d.A && d.B)), BSDMRG_EINVAL, "NULL matrix");
      BSD_CHECK(d.ldc >= d.N, BSDMRG_EINVAL, "ldc too small");
      BSD_CHECK(d.K == 0 || d.lda >= (d.transA ? d.M : d.K), BSDMRG_EINVAL, "lda too small");
      BSD_CHECK(d.K == 0 || d.ldb >= (d.transB ? d.K : d.N), BSDMRG_EINVAL, "ldb too small");
      GemmProblem g;
      g.C = tag_ptr(0, (uint64_t)d.C);
      g.ldc = d.ldc;
      g.M = d.M;
      g.N = d.N;
      g.beta = d.beta;
      if (d.K > 0) {
        GSeg sg;
        sg.A = tag_ptr(0, (uint64_t)d.A);
        sg.B = tag_ptr(0, (uint64_t)d.B);
        sg.lda = d.lda;
        sg.ldb = d.ldb;
        sg.K = d.K;
        sg.flags = (d.transA ? kTransA : 0) | (d.transB ? kTransB : 0);
        sg.alpha = d.alpha;
        g.segs.push_back(sg);
      }
      v.push_back(std::move(g));
    }
    GemmPlan plan;
    plan.build(v, precision == BSDMRG_FP64);
    GBases b{{0, 0, 0, 0}};
    plan.launch(b, S(stream), precision);
    BSD_HIP(hipStreamSynchronize(S(stream)));
  });
}

int bsdmrg_serialized_size_desc(int n, const bsdmrg_family_desc* fams, size_t* bytes) {
  return guard([&] {
    BSD_CHECK(bytes, BSDMRG_EINVAL, "NULL bytes");
    *bytes = serialized_size(desc_views(n, fams));
  });
}

int bsdmrg_pack_desc(int n, const bsdmrg_family_desc* fams, void* dst, size_t cap, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(dst, BSDMRG_EINVAL, "NULL destination");
    auto v = desc_views(n, fams);
    BSD_CHECK(cap >= serialized_size(v), BSDMRG_ENOMEM, "destination smaller than the serialized size");
    auto plan = serial_plan(v, S(stream));
    serial_pack(*plan, dst, cap, S(stream));
    BSD_HIP(hipStreamSynchronize(S(stream)));
  });
}

static_assert(sizeof(FamilyDescIn) == sizeof(bsdmrg_family_desc), "family descriptor layouts differ");
static_assert(offsetof(FamilyDescIn, data) == offsetof(bsdmrg_family_desc, data), "family descriptor layouts differ");
static_assert(offsetof(FamilyDescIn, layer_stride) == offsetof(bsdmrg_family_desc, layer_stride),
              "family descriptor layouts differ");

int bsdmrg_pack_desc_noalloc(int n, const bsdmrg_family_desc* fams, void* dst, size_t cap, bsdmrg_stream_t stream) {
  return guard([&] {
    pack_desc_noalloc(n, reinterpret_cast<const FamilyDescIn*>(fams), dst, cap, S(stream));
  });
}

int bsdmrg_noalloc_scratch_bytes(size_t* bytes) {
  return guard([&] {
    BSD_CHECK(bytes, BSDMRG_EINVAL, "NULL bytes");
    *bytes = noalloc_scratch_bytes();
  });
}

int bsdmrg_unpack_desc(int n, const bsdmrg_family_desc* fams, const void* src, size_t bytes, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(src, BSDMRG_EINVAL, "NULL source");
    auto v = desc_views(n, fams);
    BSD_CHECK(bytes == serialized_size(v), BSDMRG_ECORRUPT, "stream size does not match the families");
    auto plan = serial_plan(v, S(stream));
    serial_unpack(*plan, src, bytes, S(stream));
    int st = serial_status(*plan, S(stream));
    BSD_CHECK(st == 0, BSDMRG_ECORRUPT, "stream tables do not match the families");
  });
}

int bsdmrg_serialized_size(bsdmrg_ctx* ctx, int side, int bond, size_t* bytes) {
  return guard([&] {
    BSD_CHECK(ctx && bytes, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    *bytes = serialized_size(block_views(*b, b->left));
  });
}

int bsdmrg_pack(bsdmrg_ctx* ctx, int side, int bond, void* dst, size_t cap, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && dst, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(b->resident, BSDMRG_EBUSY, "block not resident");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    ensure_splan(*b, S(stream));
    serial_pack(*b->splan, dst, cap, S(stream));
    BSD_HIP(hipStreamSynchronize(S(stream)));
    ctx->c.st.bytes_packed += (int64_t)serial_bytes(*b->splan);
  });
}

int bsdmrg_unpack(bsdmrg_ctx* ctx, int side, int bond, const void* src, size_t bytes, bsdmrg_stream_t stream) {
  return guard([&] {
    BSD_CHECK(ctx && src, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(!b->offload_pending, BSDMRG_EBUSY, "offload in flight; wait first");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    if (!b->resident) reacquire_block(ctx->c, *b);
    ensure_splan(*b, S(stream));
    BSD_CHECK(bytes == serial_bytes(*b->splan), BSDMRG_ECORRUPT, "stream size does not match the block");
    serial_unpack(*b->splan, src, bytes, S(stream));
    int st = serial_status(*b->splan, S(stream));
    BSD_CHECK(st == 0, BSDMRG_ECORRUPT, "stream tables do not match the block");
    ctx->c.st.bytes_unpacked += (int64_t)bytes;
    ctx->c.plans.clear();
  });
}

int bsdmrg_offload(bsdmrg_ctx* ctx, int side, int bond, void* staging, void* pinned, size_t cap, int release,
                   bsdmrg_stream_t compute, bsdmrg_stream_t side_stream) {
  return guard([&] {
    BSD_CHECK(ctx && staging && pinned, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(b->resident, BSDMRG_EBUSY, "block not resident");
    BSD_CHECK(!b->offload_pending, BSDMRG_EBUSY, "previous offload still pending");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    ensure_splan(*b, S(compute));
    const size_t bytes = serial_bytes(*b->splan);
    BSD_CHECK(cap >= bytes, BSDMRG_ENOMEM, "buffers smaller than the serialized size");
    // the pack overwrites staging: after the last copy or unpack that read it
    staging_wait(ctx->c, staging, S(compute));
    serial_pack(*b->splan, staging, cap, S(compute));
    b->mark_use(S(compute));
    hipEvent_t packed;
    BSD_HIP(hipEventCreateWithFlags(&packed, hipEventDisableTiming));
    BSD_HIP(hipEventRecord(packed, S(compute)));
    BSD_HIP(hipStreamWaitEvent(S(side_stream), packed, 0));
    BSD_HIP(hipEventDestroy(packed));
    if (ctx->c.side_delay_ms > 0) delay_on(S(side_stream), ctx->c.side_delay_ms);
    BSD_HIP(hipMemcpyAsync(pinned, staging, bytes, hipMemcpyDeviceToHost, S(side_stream)));
    staging_mark(ctx->c, staging, S(side_stream));
    if (!b->offload_done) BSD_HIP(hipEventCreateWithFlags(&b->offload_done, hipEventDisableTiming));
    BSD_HIP(hipEventRecord(b->offload_done, S(side_stream)));
    b->offload_pending = true;
    b->release_after = release != 0;
    ctx->c.st.bytes_packed += (int64_t)bytes;
    ctx->c.st.bytes_d2h += (int64_t)bytes;
  });
}

int bsdmrg_offload_wait(bsdmrg_ctx* ctx, int side, int bond, double* waited) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Block* b = need_block(ctx->c, side, bond);
    auto t0 = std::chrono::steady_clock::now();
    if (b->offload_pending) BSD_HIP(hipEventSynchronize(b->offload_done));
    auto t1 = std::chrono::steady_clock::now();
    const double w = std::chrono::duration<double>(t1 - t0).count();
    if (waited) *waited = w;
    ctx->c.st.io_exposed_s += w;
    if (b->offload_pending && b->release_after) {
      // the copy has completed; products that read the block were enqueued
      // before the offload on the compute stream, which the pack followed
      b->quiesce();   // the copy, and every product enqueued before this call
      b->mem->release_physical();
      b->resident = false;
      if (!b->mem->stable()) {
        for (auto& f : b->fams) f.dev = nullptr;
        b->splan.reset();
        ctx->c.plans.clear();   // plans referencing this block are stale
      }
    }
    b->offload_pending = false;
  });
}

int bsdmrg_prefetch(bsdmrg_ctx* ctx, int side, int bond, const void* pinned, void* staging, size_t bytes,
                    bsdmrg_stream_t compute, bsdmrg_stream_t side_stream) {
  return guard([&] {
    BSD_CHECK(ctx && pinned && staging, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(!b->offload_pending, BSDMRG_EBUSY, "offload in flight; wait first");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    int st = validate_stream_host(block_views(*b, b->left), pinned, bytes);
    BSD_CHECK(st == 0, BSDMRG_ECORRUPT, "host stream does not match the block");
    if (!b->resident) reacquire_block(ctx->c, *b);
    ensure_splan(*b, S(compute));   // descriptors first: no host wait after the copy is queued
    // the copy overwrites staging: after the last pack copy-out or unpack that read it
    staging_wait(ctx->c, staging, S(side_stream));
    if (ctx->c.side_delay_ms > 0) delay_on(S(side_stream), ctx->c.side_delay_ms);
    BSD_HIP(hipMemcpyAsync(staging, pinned, bytes, hipMemcpyHostToDevice, S(side_stream)));
    hipEvent_t loaded;
    BSD_HIP(hipEventCreateWithFlags(&loaded, hipEventDisableTiming));
    BSD_HIP(hipEventRecord(loaded, S(side_stream)));
    BSD_HIP(hipStreamWaitEvent(S(compute), loaded, 0));
    BSD_HIP(hipEventDestroy(loaded));
    serial_unpack(*b->splan, staging, bytes, S(compute));
    staging_mark(ctx->c, staging, S(compute));
    if (!b->prefetch_done) BSD_HIP(hipEventCreateWithFlags(&b->prefetch_done, hipEventDisableTiming));
    BSD_HIP(hipEventRecord(b->prefetch_done, S(compute)));
    b->prefetch_pending = true;
    ctx->c.st.bytes_h2d += (int64_t)bytes;
    ctx->c.st.bytes_unpacked += (int64_t)bytes;
  });
}

int bsdmrg_segments_size(bsdmrg_ctx* ctx, int side, int bond, size_t staging_bytes, size_t* bytes,
                         int* n_segments) {
  return guard([&] {
    BSD_CHECK(ctx && bytes, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(b->resident, BSDMRG_EBUSY, "block not resident");
    ensure_splan(*b, nullptr);
    *bytes = serial_segments_size(*b->splan, staging_bytes, n_segments);
  });
}

int bsdmrg_pack_segments(bsdmrg_ctx* ctx, int side, int bond, void* staging, size_t staging_bytes, void* pinned,
                         size_t cap, size_t* written, int* n_segments, bsdmrg_stream_t compute,
                         bsdmrg_stream_t side_stream) {
  return guard([&] {
    BSD_CHECK(ctx && staging && pinned, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(b->resident, BSDMRG_EBUSY, "block not resident");
    BSD_CHECK(!b->offload_pending, BSDMRG_EBUSY, "offload in flight; wait first");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    ensure_splan(*b, S(compute));
    staging_wait(ctx->c, staging, S(compute));
    const size_t n = serial_pack_segments(*b->splan, staging, staging_bytes, pinned, cap, n_segments, S(compute),
                                          S(side_stream));
    if (written) *written = n;
    ctx->c.st.bytes_packed += (int64_t)n;
    ctx->c.st.bytes_d2h += (int64_t)n;
  });
}

int bsdmrg_unpack_segments(bsdmrg_ctx* ctx, int side, int bond, const void* pinned, size_t bytes, void* staging,
                           size_t staging_bytes, bsdmrg_stream_t compute, bsdmrg_stream_t side_stream) {
  return guard([&] {
    BSD_CHECK(ctx && staging && pinned, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    BSD_CHECK(!b->offload_pending, BSDMRG_EBUSY, "offload in flight; wait first");
    PhaseTimer tm(ctx->c, BSDMRG_PH_IO);
    const bool was_resident = b->resident;
    if (!b->resident) reacquire_block(ctx->c, *b);
    ensure_splan(*b, S(compute));
    staging_wait(ctx->c, staging, S(side_stream));
    const int st = serial_unpack_segments(*b->splan, pinned, bytes, staging, staging_bytes, S(compute),
                                          S(side_stream));
    if (st != 0 && !was_resident) {
      b->mem->release_physical();   // nothing was written: the block stays released
      b->resident = false;
    }
    BSD_CHECK(st == 0, BSDMRG_ECORRUPT, "segments do not match the block or do not cover it exactly once");
    ctx->c.st.bytes_h2d += (int64_t)bytes;
    ctx->c.st.bytes_unpacked += (int64_t)bytes;
  });
}

int bsdmrg_set_copy_workgroups(int workgroups) {
  return guard([&] {
    BSD_CHECK(workgroups >= 0, BSDMRG_EINVAL, "negative workgroup count");
    set_copy_grid(workgroups);
  });
}

int bsdmrg_prefetch_wait(bsdmrg_ctx* ctx, int side, int bond, double* waited) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Block* b = need_block(ctx->c, side, bond);
    auto t0 = std::chrono::steady_clock::now();
    if (b->prefetch_pending) BSD_HIP(hipEventSynchronize(b->prefetch_done));
    const double w = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (waited) *waited = w;
    ctx->c.st.io_exposed_s += w;
    b->prefetch_pending = false;
  });
}

int bsdmrg_set_hbm_budget(bsdmrg_ctx* ctx, size_t bytes, size_t chunk_bytes) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    ctx->c.hbm_budget = bytes;
    ctx->c.stream_chunk_bytes = chunk_bytes;
  });
}

int bsdmrg_hpsi_streamed(bsdmrg_ctx* ctx, int site, int* streamed, size_t* host_bytes, int* n_chunks) {
  return guard([&] {
    BSD_CHECK(ctx && streamed, BSDMRG_EINVAL, "NULL argument");
    auto it = ctx->c.plans.find({site, 0});
    BSD_CHECK(it != ctx->c.plans.end(), BSDMRG_ESTATE, "product not prepared");
    *streamed = it->second->stream_r ? 1 : 0;
    if (host_bytes) *host_bytes = it->second->pack_bytes;
    if (n_chunks) *n_chunks = (int)it->second->phase1.size();
  });
}

int bsdmrg_set_split_policy(bsdmrg_ctx* ctx, int fp64_heavy) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    BSD_CHECK(fp64_heavy == 0 || fp64_heavy == 1, BSDMRG_EINVAL, "policy must be 0 or 1");
    ctx->c.heavy_fp64 = fp64_heavy != 0;
  });
}

int bsdmrg_set_side_delay(bsdmrg_ctx* ctx, double ms) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    BSD_CHECK(ms >= 0.0 && ms <= 10000.0, BSDMRG_EINVAL, "delay out of [0, 10000] ms");
    ctx->c.side_delay_ms = ms;
  });
}

int bsdmrg_block_bytes(bsdmrg_ctx* ctx, int side, int bond, size_t* bytes) {
  return guard([&] {
    BSD_CHECK(ctx && bytes, BSDMRG_EINVAL, "NULL argument");
    Block* b = need_block(ctx->c, side, bond);
    *bytes = b->resident ? b->device_bytes() : 0;
  });
}

int bsdmrg_family_count(bsdmrg_ctx* ctx, int side, int bond, int* n_families, int* n_operators) {
  return guard([&] {
    BSD_CHECK(ctx, BSDMRG_EINVAL, "NULL ctx");
    Block* b = need_block(ctx->c, side, bond);
    int nop = 0;
    for (const auto& f : b->fams) nop += (int)f.keys.size();
    if (n_families) *n_families = (int)b->fams.size();
    if (n_operators) *n_operators = nop;
  });
}

int bsdmrg_stats(bsdmrg_ctx* ctx, bsdmrg_stats_t* out, int reset) {
  return guard([&] {
    BSD_CHECK(ctx && out, BSDMRG_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    std::memset(out, 0, sizeof(*out));
    for (int i = 0; i < BSDMRG_N_PHASES; ++i) out->seconds[i] = c.st.sec[i];
    out->io_exposed_s = c.st.io_exposed_s;
    out->hpsi_flops = c.st.hpsi_flops;
    out->renorm_flops = c.renorm_flops;
    out->hpsi_calls = c.st.hpsi_calls;
    out->davidson_calls = c.st.dav_calls;
    out->davidson_iters = c.st.dav_iters;
    out->truncations = c.st.truncations;
    out->renorm_steps = c.renorm_steps;
    out->bytes_packed = c.st.bytes_packed;
    out->bytes_unpacked = c.st.bytes_unpacked;
    out->bytes_d2h = c.st.bytes_d2h;
    out->bytes_h2d = c.st.bytes_h2d;
    if (reset) {
      c.st = Ctx::Stats();
      c.renorm_flops = 0.0;
      c.renorm_wall_s = 0.0;
      c.renorm_dev_s = 0.0;
      c.renorm_steps = 0;
    }
  });
}

}  // extern "C"
