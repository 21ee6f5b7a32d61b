// Renormalized block operators on the device and the renormalization step
// (Sec. II.B: the enlarged block's operators are mapped to the new basis and
// kept for later steps).  Operators of one block that share a quantum-number
// change dq share one skeleton and live as layers of one family (Fig. 4a).
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include "ctx.h"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <system_error>
#include <thread>
#include <unordered_map>

namespace bsd {

DevBuf::~DevBuf() { release(); }
void DevBuf::reserve(size_t bytes) {
  if (bytes <= n && p) return;
  release();
  if (bytes == 0) bytes = 256;
  BSD_HIP(hipMalloc(&p, bytes));
  n = bytes;
}
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  n = 0;
}

Ctx::~Ctx() {
  for (auto& kv : staging_busy) (void)hipEventDestroy(kv.second);
}

void Block::mark_use(hipStream_t s) {
  if (!last_use) BSD_HIP(hipEventCreateWithFlags(&last_use, hipEventDisableTiming));
  BSD_HIP(hipEventRecord(last_use, s));
}

void Block::quiesce() {
  if (offload_pending && offload_done) (void)hipEventSynchronize(offload_done);
  if (prefetch_pending && prefetch_done) (void)hipEventSynchronize(prefetch_done);
  if (last_use) (void)hipEventSynchronize(last_use);
}

Block::~Block() {
  // no queued copy, unpack or product may touch the memory after it is freed
  quiesce();
  if (offload_done) (void)hipEventDestroy(offload_done);
  if (prefetch_done) (void)hipEventDestroy(prefetch_done);
  if (last_use) (void)hipEventDestroy(last_use);
}

static hipMemAllocationProp device_prop(int dev) {
  hipMemAllocationProp prop = {};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = dev;
  return prop;
}

static void vmm_note(const char* what, hipError_t e, size_t at, size_t total) {
  if (std::getenv("BSDMRG_VERBOSE"))
    std::fprintf(stderr, "bsdmrg: %s failed (%s) at byte %zu of %zu; block memory falls back\n", what,
                 hipGetErrorString(e), at, total);
}

void BlockMem::create(size_t n) {
  bytes = std::max<size_t>(n, 256);
  BSD_HIP(hipGetDevice(&device));
  int vmm_ok = 0;
  if (hipDeviceGetAttribute(&vmm_ok, hipDeviceAttributeVirtualMemoryManagementSupported, device) != hipSuccess)
    vmm_ok = 0;
  size_t gran = 0;
  if (vmm_ok) {
    hipMemAllocationProp prop = device_prop(device);
    // the recommended granularity (2 MiB pages): access rights are set on
    // whole pages, and a range whose end is not page aligned is refused
    if (hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityRecommended) != hipSuccess || gran == 0)
      vmm_ok = 0;
  }
  if (vmm_ok) {
    reserved = (bytes + gran - 1) / gran * gran;
    // physical memory in pieces of at most 1 GiB, mapped back to back
    piece = std::min(reserved, std::max(gran, ((size_t)1 << 30) / gran * gran));
    const hipError_t e = hipMemAddressReserve(&va, reserved, 0, nullptr, 0);
    if (e != hipSuccess) {
      vmm_note("hipMemAddressReserve", e, 0, reserved);
      va = nullptr;
      vmm_ok = 0;
    } else {
      vmm = true;
      if (!map_pieces()) {
        // fall back to a plain allocation (its address is not stable)
        (void)hipMemAddressFree(va, reserved);
        va = nullptr;
        vmm = false;
        vmm_ok = 0;
      }
    }
  }
  if (!vmm_ok) {
    if (std::getenv("BSDMRG_VERBOSE")) std::fprintf(stderr, "bsdmrg: block of %zu bytes in plain memory\n", bytes);
    vmm = false;
    reserved = bytes;
    BSD_HIP(hipMalloc(&va, reserved));
    mapped = true;
  }
}

bool BlockMem::map_pieces() {
  hipMemAllocationProp prop = device_prop(device);
  hipMemAccessDesc ad = {};
  ad.location = prop.location;
  ad.flags = hipMemAccessFlagsProtReadWrite;
  handles.clear();
  size_t done = 0;
  bool ok = true;
  while (done < reserved) {
    const size_t len = std::min(piece, reserved - done);
    hipMemGenericAllocationHandle_t h;
    hipError_t e = hipMemCreate(&h, len, &prop, 0);
    if (e != hipSuccess) {
      vmm_note("hipMemCreate", e, done, reserved);
      ok = false;
      break;
    }
    char* at = static_cast<char*>(va) + done;
    e = hipMemMap(at, len, 0, h, 0);
    if (e != hipSuccess) {
      vmm_note("hipMemMap", e, done, reserved);
      (void)hipMemRelease(h);
      ok = false;
      break;
    }
    handles.push_back(reinterpret_cast<uint64_t>(h));
    done += len;
  }
  if (ok) {
    // access for the whole range at once, after every piece is mapped
    const hipError_t e = hipMemSetAccess(va, reserved, &ad, 1);
    if (e != hipSuccess) {
      vmm_note("hipMemSetAccess", e, 0, reserved);
      ok = false;
    }
  }
  if (!ok) {
    size_t off = 0;
    for (size_t i = 0; i < handles.size(); ++i) {
      const size_t len = std::min(piece, reserved - off);
      (void)hipMemUnmap(static_cast<char*>(va) + off, len);
      (void)hipMemRelease(reinterpret_cast<hipMemGenericAllocationHandle_t>(handles[i]));
      off += len;
    }
    handles.clear();
    (void)hipGetLastError();
    return false;
  }
  mapped = true;
  return true;
}

void BlockMem::acquire_physical() {
  if (mapped) return;
  if (!vmm) {
    BSD_HIP(hipMalloc(&va, reserved));
    mapped = true;
    return;
  }
  BSD_CHECK(map_pieces(), 4, "device memory for the block could not be created again");
}

void BlockMem::release_physical() {
  if (!mapped) return;
  if (!vmm) {
    (void)hipFree(va);
    va = nullptr;
    mapped = false;
    return;
  }
  size_t off = 0;
  for (size_t i = 0; i < handles.size(); ++i) {
    const size_t len = std::min(piece, reserved - off);
    (void)hipMemUnmap(static_cast<char*>(va) + off, len);
    (void)hipMemRelease(reinterpret_cast<hipMemGenericAllocationHandle_t>(handles[i]));
    off += len;
  }
  handles.clear();
  mapped = false;
}

BlockMem::~BlockMem() {
  release_physical();
  if (vmm && va) (void)hipMemAddressFree(va, reserved);
}

Skeleton make_skeleton(const Basis& in, const Basis& out, const Q& dq) {
  Skeleton sk;
  sk.dq = dq;
  sk.by_in.assign(in.q.size(), -1);
  int64_t off = 0;
  for (int i = 0; i < (int)in.q.size(); ++i) {
    int j = out.find(in.q[i] + dq);
    if (j < 0) continue;
    SkBlock b;
    b.in = i;
    b.out = j;
    b.rows = out.dim[j];
    b.cols = in.dim[i];
    b.ld = (b.cols + 1) & ~1;
    b.off = off;
    off += (int64_t)b.rows * b.ld;
    sk.by_in[i] = (int)sk.blocks.size();
    sk.blocks.push_back(b);
  }
  sk.layer_stride = (off + 31) / 32 * 32;
  return sk;
}

const double* Block::op_block(const OpKey& k, int in_idx, int* rows, int* cols, int* ld) const {
  auto it = ops.find(k);
  if (it == ops.end()) return nullptr;
  const Family& f = fams[it->second.fam];
  int b = f.sk.by_in[in_idx];
  if (b < 0) return nullptr;
  const SkBlock& sb = f.sk.blocks[b];
  *rows = sb.rows;
  *cols = sb.cols;
  *ld = sb.ld;
  return f.dev + (int64_t)it->second.layer * f.sk.layer_stride + sb.off;
}

size_t Block::device_bytes() const {
  size_t s = 0;
  for (auto& f : fams) s += f.bytes();
  return s;
}

static std::vector<OpKey> block_keys(bool left, int first, int last, int L, bool normal) {
  std::vector<OpKey> k;
  const int NM = 2 * L;
  auto add = [&](char c, int p, int q) {
    OpKey o;
    o.kind = c;
    o.p = p;
    o.q = q;
    k.push_back(o);
  };
  if (left) {
    const int nm = 2 * last;
    if (last > 0) add('H', -1, -1);
    for (int p = 0; p < nm; ++p) add('c', p, -1);
    for (int p = 0; p < nm; ++p)
      for (int q = p + 1; q < nm; ++q) add('A', p, q);
    for (int p = 0; p < nm; ++p)
      for (int q = 0; q < nm; ++q) add('B', p, q);
    for (int y = nm; y < NM; ++y) add('S', y, -1);
  } else if (normal) {
    // normal operators of the block's own modes (the smaller side)
    const int m0 = 2 * first;
    if (first < L) add('H', -1, -1);
    for (int r = m0; r < NM; ++r) add('c', r, -1);
    for (int x = 0; x < m0; ++x) add('S', x, -1);
    for (int p = m0; p < NM; ++p)
      for (int q = p + 1; q < NM; ++q) add('A', p, q);
    for (int p = m0; p < NM; ++p)
      for (int q = m0; q < NM; ++q) add('B', p, q);
  } else {
    const int m0 = 2 * first;
    if (first < L) add('H', -1, -1);
    for (int r = m0; r < NM; ++r) add('c', r, -1);
    for (int x = 0; x < m0; ++x) add('S', x, -1);
    for (int p = 0; p < m0; ++p)
      for (int q = p + 1; q < m0; ++q) add('P', p, q);
    for (int p = 0; p < m0; ++p)
      for (int q = 0; q < m0; ++q) add('Q', p, q);
  }
  return k;
}

static std::unique_ptr<Block> alloc_block(bool left, int first, int last, const Basis& basis,
                                          const std::vector<OpKey>& keys, hipStream_t s) {
  auto B = std::make_unique<Block>();
  B->left = left;
  B->first = first;
  B->last = last;
  B->basis = basis;
  std::map<Q, int> famidx;
  for (const auto& k : keys) {
    Q dq = key_dq(k, left);
    auto it = famidx.find(dq);
    int f;
    if (it == famidx.end()) {
      f = (int)B->fams.size();
      famidx[dq] = f;
      Family fam;
      fam.sk = make_skeleton(basis, basis, dq);
      B->fams.push_back(std::move(fam));
    } else {
      f = it->second;
    }
    OpRef r;
    r.fam = f;
    r.layer = (int)B->fams[f].keys.size();
    B->fams[f].keys.push_back(k);
    B->ops[k] = r;
  }
  size_t total = 0;
  for (auto& f : B->fams) {
    B->fam_off.push_back(total);
    total += (f.bytes() + 255) / 256 * 256;
  }
  B->mem = std::make_unique<BlockMem>();
  B->mem->create(total);
  if (total) BSD_HIP(hipMemsetAsync(B->mem->va, 0, total, s));
  for (size_t i = 0; i < B->fams.size(); ++i)
    B->fams[i].dev = reinterpret_cast<double*>(static_cast<char*>(B->mem->va) + B->fam_off[i]);
  return B;
}

void make_vacuum_blocks(Ctx& ctx) {
  auto l = std::make_unique<Block>();
  l->left = true;
  l->first = l->last = 0;
  l->basis.add({0, 0}, 1);
  ctx.left[0] = std::move(l);
  auto r = std::make_unique<Block>();
  r->left = false;
  r->first = r->last = ctx.L;
  r->basis.add({0, 0}, 1);
  ctx.right[ctx.L] = std::move(r);
}

Block* get_block(Ctx& ctx, bool left, int bond) {
  auto& m = left ? ctx.left : ctx.right;
  auto it = m.find(bond);
  if (it == m.end()) return nullptr;
  return it->second.get();
}

// ---------------------------------------------------------------- renormalization
namespace {

Q local_dq(const Mat& M, const SiteSet& C) {
  for (int i = 0; i < M.n; ++i)
    for (int j = 0; j < M.n; ++j)
      if (M(i, j) != 0.0) return C.q[i] - C.q[j];
  return {0, 0};
}

// block-side operator of a group: a stored op, the identity, or an aggregate
struct Ref {
  int kind;        // 0 stored op, 1 identity, 2 aggregate
  OpKey key;
  bool trans = false;
  int agg = -1;    // index into aggregates
  Q dq;
};

struct AggOp {
  Skeleton sk;
  std::vector<Term> terms;
};

// Pointer to block (in_idx -> out) of op(ref), with its storage orientation.
struct Operand {
  const double* p = nullptr;
  int64_t ld = 0;
  bool trans = false;
  bool ident = false;
  int rows = 0, cols = 0;   // of op(ref) block
};

}  // namespace

static Operand ref_block(const Block& blk, const Ref& r, const AggOp* agg, const double* agg_base,
                         int in_idx) {
  Operand o;
  const Basis& bs = blk.basis;
  Q qout = bs.q[in_idx] + r.dq;
  int out_idx = bs.find(qout);
  if (out_idx < 0) return o;
  if (r.kind == 1) {
    o.ident = true;
    o.rows = o.cols = bs.dim[in_idx];
    o.p = nullptr;  // unused
    return o;
  }
  if (r.kind == 2) {
    const AggOp& a = *agg;
    int b = a.sk.by_in[in_idx];
    if (b < 0) return o;
    const SkBlock& sb = a.sk.blocks[b];
    o.p = agg_base + sb.off;
    o.ld = sb.ld;
    o.rows = sb.rows;
    o.cols = sb.cols;
    return o;
  }
  int rr, cc, ld;
  if (!r.trans) {
    const double* p = blk.op_block(r.key, in_idx, &rr, &cc, &ld);
    if (!p) return o;
    o.p = p;
    o.ld = ld;
    o.rows = rr;
    o.cols = cc;
  } else {
    // op(O) = O^T maps in -> out, so O maps out -> in
    const double* p = blk.op_block(r.key, out_idx, &rr, &cc, &ld);
    if (!p) return o;
    o.p = p;
    o.ld = ld;
    o.trans = true;
    o.rows = cc;
    o.cols = rr;
  }
  return o;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static void renormalize(Ctx& ctx, bool left, int bond, hipStream_t s) {
  BSD_CHECK(ctx.have_ints, 1, "integrals not loaded");
  const double t_start = now_s();
  const int L = ctx.L, NM = 2 * L;
  Block* old = get_block(ctx, left, bond);
  BSD_CHECK(old != nullptr, 1, "source block missing");
  const int site = left ? bond : bond - 1;
  BSD_CHECK(site >= 0 && site < L, 1, "site out of range");
  const SiteTensor& T = ctx.sites[site];
  BSD_CHECK(T.set, 1, "site tensor not set");
  const SiteSet S = make_siteset(site, 1);

  // new basis (electrons inside the new block) and map site-tensor blocks
  Basis nb;
  {
    std::vector<std::pair<Q, int>> v;
    const Basis& src = left ? T.right : T.left;
    for (size_t i = 0; i < src.q.size(); ++i)
      v.push_back({left ? src.q[i] : ctx.target - src.q[i], src.dim[i]});
    std::sort(v.begin(), v.end(), [](auto& a, auto& b) { return a.first < b.first; });
    for (auto& x : v) nb.add(x.first, x.second);
  }
  // old block basis must match the tensor's other bond
  {
    const Basis& other = left ? T.left : T.right;
    for (size_t i = 0; i < other.q.size(); ++i) {
      Q lab = left ? other.q[i] : ctx.target - other.q[i];
      int j = old->basis.find(lab);
      BSD_CHECK(j >= 0 && old->basis.dim[j] == other.dim[i], 3, "site tensor does not match block basis");
    }
  }
  // site tensor block for (old sector idx, s) with its new sector idx
  struct TB {
    const double* p = nullptr;
    int rows = 0, cols = 0, nidx = -1;
  };
  auto tblock = [&](int old_idx, int sstate) -> TB {
    TB r;
    Q qo = old->basis.q[old_idx];
    if (left) {
      int l = T.left.find(qo);
      if (l < 0) return r;
      auto it = T.by_ls.find({l, sstate});
      if (it == T.by_ls.end()) return r;
      const auto& b = T.blocks[it->second];
      r.p = T.ptr(it->second);
      r.rows = b.rows;
      r.cols = b.cols;
      r.nidx = nb.find(qo + kSiteQ[sstate]);
    } else {
      // old R label qo; new label qn = qo + q_s; tensor left bond label = target - qn
      Q qn = qo + kSiteQ[sstate];
      int l = T.left.find(ctx.target - qn);
      if (l < 0) return r;
      auto it = T.by_ls.find({l, sstate});
      if (it == T.by_ls.end()) return r;
      const auto& b = T.blocks[it->second];
      r.p = T.ptr(it->second);
      r.rows = b.rows;   // d_new
      r.cols = b.cols;   // d_R
      r.nidx = nb.find(qn);
    }
    return r;
  };

  const int nfirst = left ? 0 : site, nlast = left ? site + 1 : L;
  // a right block at a bond at or beyond right_normal_from keeps normal
  // operators; its source must then be normal too (or the vacuum)
  const bool normal = !left && site >= ctx.right_normal_from;
  BSD_CHECK(!normal || old->normal || old->first == L, 2,
            "a right block with normal operators needs a normal (or vacuum) source block");
  std::vector<OpKey> keys = block_keys(left, nfirst, nlast, L, normal);
  auto nw = alloc_block(left, nfirst, nlast, nb, keys, s);
  nw->normal = normal;

  // expansions and block-side references
  std::vector<Ref> refs;
  std::map<std::tuple<int, char, int, int, bool>, int> ref_index;  // stored/identity refs
  std::vector<AggOp> aggs;
  struct GRef {
    int ref;
    double coef;
    Mat M;
    int mpar;
  };
  std::vector<std::vector<GRef>> per_key(keys.size());
  for (size_t ki = 0; ki < keys.size(); ++ki) {
    const OpKey& k = keys[ki];
    std::vector<Group> gs = left ? expand_left(k, 2 * site, S, ctx.ints)
                                 : expand_right(k, S, 2 * (site + 1), NM, ctx.ints, old->normal || old->first == L);
    const Q kdq = key_dq(k, left);
    for (auto& g : gs) {
      Q ldq = local_dq(g.M, S);
      Q bdq = kdq - ldq;
      int mpar = ldq.parity();
      GRef gr;
      gr.M = g.M;
      gr.mpar = mpar;
      if (g.terms.size() == 1) {
        const Term& t = g.terms[0];
        Ref r;
        r.kind = t.key.kind == 'I' ? 1 : 0;
        r.key = t.key;
        r.trans = t.trans;
        Q tdq = t.key.kind == 'I' ? Q{0, 0} : key_dq(t.key, left);
        if (t.trans) tdq = -tdq;
        BSD_CHECK(tdq == bdq, 1, "inconsistent dq in expansion");
        if (r.kind == 0 && old->ops.find(t.key) == old->ops.end()) continue;
        r.dq = bdq;
        auto id = std::make_tuple(r.kind, t.key.kind, t.key.p, t.key.q, t.trans);
        auto it = ref_index.find(id);
        if (it == ref_index.end()) {
          ref_index[id] = (int)refs.size();
          gr.ref = (int)refs.size();
          refs.push_back(r);
        } else {
          gr.ref = it->second;
        }
        gr.coef = t.coef;
      } else {
        AggOp a;
        a.sk = make_skeleton(old->basis, old->basis, bdq);
        for (const auto& t : g.terms) {
          Q tdq = t.key.kind == 'I' ? Q{0, 0} : key_dq(t.key, left);
          if (t.trans) tdq = -tdq;
          BSD_CHECK(tdq == bdq, 1, "inconsistent dq in aggregate");
          if (t.key.kind != 'I' && old->ops.find(t.key) == old->ops.end()) continue;
          a.terms.push_back(t);
        }
        if (a.terms.empty()) continue;
        Ref r;
        r.kind = 2;
        r.agg = (int)aggs.size();
        r.dq = bdq;
        aggs.push_back(std::move(a));
        gr.ref = (int)refs.size();
        refs.push_back(r);
        gr.coef = 1.0;
      }
      per_key[ki].push_back(std::move(gr));
    }
  }

  // phase-1 intermediates T(ref, s, old sector): op(ref) applied to the site tensor
  struct TKey {
    int ref, sstate, oidx;
    bool operator<(const TKey& o) const {
      return std::tie(ref, sstate, oidx) < std::tie(o.ref, o.sstate, o.oidx);
    }
  };
  struct TVal {
    int64_t off;     // -1: identity (use the site tensor block directly)
    int rows, cols;  // T rows x cols (ld = cols)
  };
  // which (ref, s) pairs are needed, and each ref's intermediates
  std::map<std::pair<int, int>, bool> need;
  for (auto& v : per_key)
    for (auto& gr : v)
      for (int sp = 0; sp < 4; ++sp)
        for (int s0 = 0; s0 < 4; ++s0)
          if (gr.M(sp, s0) != 0.0) need[{gr.ref, s0}] = true;
  std::vector<std::vector<std::pair<TKey, TVal>>> ref_t(refs.size());
  std::vector<int64_t> ref_cost(refs.size(), 0);   // workspace elements of a ref (aggregate + its T)
  for (auto& nd : need) {
    int ri = nd.first.first, s0 = nd.first.second;
    const Ref& r = refs[ri];
    for (int oi = 0; oi < (int)old->basis.q.size(); ++oi) {
      TB tb = tblock(oi, s0);
      if (!tb.p || tb.nidx < 0) continue;
      int oo = old->basis.find(old->basis.q[oi] + r.dq);
      if (oo < 0) continue;
      if (r.kind == 1) {
        ref_t[ri].push_back({{ri, s0, oi}, {-1, 0, 0}});
        continue;
      }
      // does op(ref) have a block at oi?
      if (r.kind == 2) {
        if (aggs[r.agg].sk.by_in[oi] < 0) continue;
      } else {
        int rr, cc, ld;
        int src = r.trans ? oo : oi;
        if (!old->op_block(r.key, src, &rr, &cc, &ld)) continue;
      }
      const int trows = old->basis.dim[oo];
      const int tcols = left ? tb.cols : tb.rows;  // d_new
      ref_t[ri].push_back({{ri, s0, oi}, {0, trows, tcols}});
      ref_cost[ri] += ((int64_t)trows * tcols + 1) / 2 * 2;
    }
  }
  for (size_t ri = 0; ri < refs.size(); ++ri)
    if (refs[ri].kind == 2) ref_cost[ri] += aggs[refs[ri].agg].sk.layer_stride;

  // output operators in batches whose workspace (aggregates + intermediates of
  // the refs they use) stays under the budget; a ref shared by two batches is
  // computed in both
  struct Batch {
    size_t k0 = 0, k1 = 0;
    std::vector<int> refs;
    DevBuf tasks, terms;   // aggregation lists
    int ntasks = 0;
    GemmPlan p1, p2;       // phase 1 and phase 2 tile lists
    bool has_p1 = false, has_p2 = false;
    bool ready = false;
    std::exception_ptr err;
  };
  const int64_t budget = (int64_t)(ctx.renorm_ws_budget / sizeof(double));
  // at least two batches per planning thread where the budget allows fewer
  const int max_threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t max_keys = std::max<size_t>(1, (keys.size() + 2 * max_threads - 1) / (2 * max_threads));
  std::vector<std::unique_ptr<Batch>> batches;
  int64_t ws_max = 1;
  for (size_t k0 = 0; k0 < keys.size();) {
    auto B = std::make_unique<Batch>();
    std::vector<char> in_batch(refs.size(), 0);
    int64_t bws = 0;
    size_t k1 = k0;
    for (; k1 < keys.size(); ++k1) {
      int64_t add = 0;
      for (const auto& gr : per_key[k1])
        if (!in_batch[gr.ref]) add += ref_cost[gr.ref];
      if (k1 > k0 && (bws + add > budget || k1 - k0 >= max_keys)) break;
      for (const auto& gr : per_key[k1])
        if (!in_batch[gr.ref]) {
          in_batch[gr.ref] = 1;
          B->refs.push_back(gr.ref);
        }
      bws += add;
    }
    B->k0 = k0;
    B->k1 = k1;
    ws_max = std::max(ws_max, bws);
    batches.push_back(std::move(B));
    k0 = k1;
  }
  ctx.ws.reserve(ws_max * sizeof(double));
  double* const ws = static_cast<double*>(ctx.ws.p);

  // host lists of one batch (run by the planning threads; reads shared state only)
  auto plan_batch = [&](Batch& bt, hipStream_t up) {
    // batch-local workspace offsets of the aggregates and intermediates
    std::unordered_map<int, int64_t> agg_off;
    std::map<TKey, TVal> tmap;
    int64_t ws_elems = 0;
    for (int ri : bt.refs) {
      if (refs[ri].kind == 2) {
        agg_off[refs[ri].agg] = ws_elems;
        ws_elems += aggs[refs[ri].agg].sk.layer_stride;
      }
      for (auto tv : ref_t[ri]) {
        if (tv.second.off >= 0) {
          tv.second.off = ws_elems;
          ws_elems += ((int64_t)tv.second.rows * tv.second.cols + 1) / 2 * 2;
        }
        tmap[tv.first] = tv.second;
      }
    }
    BSD_CHECK(ws_elems <= ws_max, 1, "renormalization workspace bookkeeping");
    auto agg_base = [&](const Ref& r) -> const double* {
      return r.kind == 2 ? ws + agg_off.at(r.agg) : nullptr;
    };

    // aggregation
    std::vector<AggTask> tasks;
    std::vector<AggTerm> terms;
    std::vector<const OpRef*> term_op;
    for (int ri : bt.refs) {
      if (refs[ri].kind != 2) continue;
      const AggOp& a = aggs[refs[ri].agg];
      double* base = ws + agg_off.at(refs[ri].agg);
      // each term's stored operator, looked up once
      term_op.assign(a.terms.size(), nullptr);
      for (size_t ti = 0; ti < a.terms.size(); ++ti)
        if (a.terms[ti].key.kind != 'I') {
          auto it = old->ops.find(a.terms[ti].key);
          if (it != old->ops.end()) term_op[ti] = &it->second;
        }
      for (const auto& sb : a.sk.blocks) {
        AggTask t;
        t.out = base + sb.off;
        t.ldo = sb.ld;
        t.rows = sb.rows;
        t.cols = sb.cols;
        t.t0 = (int)terms.size();
        for (size_t ti = 0; ti < a.terms.size(); ++ti) {
          const Term& tm = a.terms[ti];
          AggTerm x;
          x.coef = tm.coef;
          x.pad = 0;
          if (tm.key.kind == 'I') {
            if (sb.in != sb.out) continue;
            x.in = nullptr;
            x.ldi = 0;
            x.flags = kIdentA;
          } else {
            if (!term_op[ti]) continue;
            const Family& f = old->fams[term_op[ti]->fam];
            const int b = f.sk.by_in[tm.trans ? sb.out : sb.in];
            if (b < 0) continue;
            const SkBlock& ob = f.sk.blocks[b];
            x.in = f.dev + (int64_t)term_op[ti]->layer * f.sk.layer_stride + ob.off;
            x.ldi = ob.ld;
            x.flags = tm.trans ? kTransA : 0;
          }
          terms.push_back(x);
        }
        t.nt = (int)terms.size() - t.t0;
        int ntrans = 0;
        for (int k = t.t0; k < t.t0 + t.nt; ++k) ntrans += (terms[k].flags & kTransA) ? 1 : 0;
        t.col_major = 2 * ntrans > t.nt ? 1 : 0;
        t.pad = 0;
        tasks.push_back(t);
      }
    }
    if (!tasks.empty()) {
      bt.tasks.reserve(tasks.size() * sizeof(AggTask));
      bt.terms.reserve(std::max<size_t>(1, terms.size()) * sizeof(AggTerm));
      BSD_HIP(hipMemcpyAsync(bt.tasks.p, tasks.data(), tasks.size() * sizeof(AggTask), hipMemcpyHostToDevice, up));
      if (!terms.empty())
        BSD_HIP(hipMemcpyAsync(bt.terms.p, terms.data(), terms.size() * sizeof(AggTerm), hipMemcpyHostToDevice, up));
      BSD_HIP(hipStreamSynchronize(up));
      bt.ntasks = (int)tasks.size();
    }
    GemmBuildOpts opts;
    opts.upload = up;

    // phase 1: T = op(ref) X, X = A_s (left) or B_s^T (right)
    std::vector<GemmProblem> p1;
    for (auto& kv : tmap) {
      if (kv.second.off < 0) continue;
      const TKey& tk = kv.first;
      const Ref& r = refs[tk.ref];
      Operand o = ref_block(*old, r, r.kind == 2 ? &aggs[r.agg] : nullptr, agg_base(r), tk.oidx);
      TB tb = tblock(tk.oidx, tk.sstate);
      GemmProblem gp;
      gp.C = tag_ptr(0, (uint64_t)(ws + kv.second.off));
      gp.ldc = kv.second.cols;
      gp.M = kv.second.rows;
      gp.N = kv.second.cols;
      gp.beta = 0.0;
      GSeg sg;
      sg.alpha = 1.0;
      sg.K = o.cols;
      sg.flags = (o.trans ? kTransA : 0) | (o.ident ? kIdentA : 0);
      sg.A = tag_ptr(0, (uint64_t)o.p);
      sg.lda = o.ld;
      sg.B = tag_ptr(0, (uint64_t)tb.p);
      if (left) {
        sg.ldb = tb.cols;     // A_s: d_old x d_new
      } else {
        sg.flags |= kTransB;  // B_s: d_new x d_old, used transposed
        sg.ldb = tb.cols;
      }
      gp.segs.push_back(sg);
      p1.push_back(std::move(gp));
    }
    if (!p1.empty()) {
      bt.p1.build(p1, opts);
      bt.has_p1 = true;
    }

    // phase 2: new op blocks of the batch's keys
    std::vector<GemmProblem> p2;
    for (size_t ki = bt.k0; ki < bt.k1; ++ki) {
      const OpRef& orf = nw->ops.at(keys[ki]);
      const Family& fam = nw->fams[orf.fam];
      for (const auto& sb : fam.sk.blocks) {
        GemmProblem gp;
        gp.C = tag_ptr(0, (uint64_t)(fam.dev + (int64_t)orf.layer * fam.sk.layer_stride + sb.off));
        gp.ldc = sb.ld;
        gp.M = sb.rows;
        gp.N = sb.cols;
        gp.beta = 0.0;
        const Q qn = nb.q[sb.in];
        for (const auto& gr : per_key[ki]) {
          const Ref& r = refs[gr.ref];
          for (int s0 = 0; s0 < 4; ++s0) {
            const Q qo = qn - kSiteQ[s0];
            int oi = old->basis.find(qo);
            if (oi < 0) continue;
            auto it = tmap.find({gr.ref, s0, oi});
            if (it == tmap.end()) continue;
            int oo = old->basis.find(qo + r.dq);
            for (int sp = 0; sp < 4; ++sp) {
              double m = gr.M(sp, s0);
              if (m == 0.0) continue;
              if (old->basis.q[oo] + kSiteQ[sp] != nb.q[sb.out]) continue;
              TB to = tblock(oo, sp);
              if (!to.p) continue;
              double sign;
              if (left) sign = (gr.mpar && old->basis.q[oi].parity()) ? -1.0 : 1.0;
              else sign = (r.dq.parity() && kSiteQ[s0].parity()) ? -1.0 : 1.0;
              GSeg sg;
              sg.alpha = gr.coef * m * sign;
              sg.K = old->basis.dim[oo];
              if (left) {
                sg.A = tag_ptr(0, (uint64_t)to.p);    // A_{s'}: d_old' x d_new', used transposed
                sg.lda = to.cols;
                sg.flags = kTransA;
              } else {
                sg.A = tag_ptr(0, (uint64_t)to.p);    // B_{s'}: d_new' x d_old'
                sg.lda = to.cols;
                sg.flags = 0;
              }
              if (it->second.off >= 0) {
                sg.B = tag_ptr(0, (uint64_t)(ws + it->second.off));
                sg.ldb = it->second.cols;
              } else {
                TB ti = tblock(oi, s0);
                sg.B = tag_ptr(0, (uint64_t)ti.p);
                sg.ldb = ti.cols;
                if (!left) sg.flags |= kTransB;
              }
              gp.segs.push_back(sg);
            }
          }
        }
        if (!gp.segs.empty()) p2.push_back(std::move(gp));
      }
    }
    if (!p2.empty()) {
      bt.p2.build(p2, opts);
      bt.has_p2 = true;
    }
  };

  // Batches are planned by a pool of host threads, each copying its lists on
  // a stream of its own, and launched in order on `s` as they become ready, so
  // that the planning of later batches overlaps the device work of earlier
  // ones.  Every batch reuses the one workspace: stream order serializes them.
  // The lists stay allocated until the step's final synchronization.
  const int nthreads = (int)std::min<size_t>(batches.size(), max_threads);
  std::vector<hipStream_t> ups(nthreads, nullptr);
  for (auto& u : ups) BSD_HIP(hipStreamCreateWithFlags(&u, hipStreamNonBlocking));
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<size_t> next{0};
  std::atomic<bool> stop{false};
  std::vector<std::thread> pool;
  int dev = 0;
  BSD_HIP(hipGetDevice(&dev));
  for (int t = 0; t < nthreads; ++t) {
    try {
      pool.emplace_back([&, t] {
        (void)hipSetDevice(dev);   // a failure shows in the batch's own HIP calls
        for (;;) {
          const size_t i = next.fetch_add(1);
          if (i >= batches.size() || stop.load()) return;
          Batch& bt = *batches[i];
          try {
            plan_batch(bt, ups[t]);
          } catch (...) {
            bt.err = std::current_exception();
          }
          {
            std::lock_guard<std::mutex> lk(mu);
            bt.ready = true;
          }
          cv.notify_all();
        }
      });
    } catch (const std::system_error&) {
      break;   // fewer planning threads: the running ones take every batch
    }
  }
  if (pool.empty() && !batches.empty()) {
    for (auto u : ups) (void)hipStreamDestroy(u);
    BSD_CHECK(false, 4, "could not start a planning thread");
  }
  std::vector<hipEvent_t> evs(2 * batches.size(), nullptr);
  std::exception_ptr failure;
  double fl = 0.0;
  try {
    for (auto& e : evs) BSD_HIP(hipEventCreate(&e));
    for (size_t i = 0; i < batches.size(); ++i) {
      Batch& bt = *batches[i];
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return bt.ready; });
      }
      if (bt.err) std::rethrow_exception(bt.err);
      GBases b{{0, 0, 0, 0}};
      BSD_HIP(hipEventRecord(evs[2 * i], s));
      if (bt.ntasks > 0)
        launch_aggregate((const AggTask*)bt.tasks.p, (const AggTerm*)bt.terms.p, bt.ntasks, s);
      if (bt.has_p1) {
        bt.p1.launch(b, s);
        fl += bt.p1.flops;
      }
      if (bt.has_p2) {
        bt.p2.launch(b, s);
        fl += bt.p2.flops;
      }
      BSD_HIP(hipEventRecord(evs[2 * i + 1], s));
    }
  } catch (...) {
    failure = std::current_exception();
    stop = true;
  }
  for (auto& th : pool) th.join();
  (void)hipStreamSynchronize(s);
  double t_dev = 0.0;
  if (!failure)
    for (size_t i = 0; i < batches.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, evs[2 * i], evs[2 * i + 1]) == hipSuccess) t_dev += ms * 1e-3;
    }
  for (auto e : evs)
    if (e) (void)hipEventDestroy(e);
  for (auto u : ups) (void)hipStreamDestroy(u);
  if (failure) std::rethrow_exception(failure);
  BSD_HIP(hipGetLastError());
  ctx.renorm_flops += fl;
  ctx.renorm_dev_s += t_dev;
  ctx.renorm_wall_s += now_s() - t_start;
  ctx.renorm_steps += 1;
  auto& m = left ? ctx.left : ctx.right;
  m[left ? bond + 1 : bond - 1] = std::move(nw);
}

void renormalize_left_block(Ctx& ctx, int bond, hipStream_t s) { renormalize(ctx, true, bond, s); }
void renormalize_right_block(Ctx& ctx, int bond, hipStream_t s) { renormalize(ctx, false, bond, s); }

}  // namespace bsd
