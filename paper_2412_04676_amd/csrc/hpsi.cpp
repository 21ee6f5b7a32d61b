// Effective-Hamiltonian product H.psi for the two-site superblock L . C . R
// (C = sites i, i+1 treated exactly; Sec. II.B step 2).
//
// The Hamiltonian is split as X = L . C | Y = R with the partition rule of the
// operator algebra, so every term is (operator on L . C) (x) (operator on R).
// Operators on R are the stored complementary set (or the identity); the
// operator on L . C of each R "channel" is expanded into groups
// (aggregated L operator) (x) (16 x 16 matrix on C).  With psi stored as one
// tall matrix per right sector (all (q_l, c) blocks stacked), each channel b is
//   phase 1:  V_b = Psi R_b^T                  (one GEMM per right sector)
//   phase 2:  Phi[l', c', r'] += sum alpha Lambda[l' <- l] V_b[(l, c), r']
// where phase 2 concatenates the K dimension over all channels, groups and
// local transitions c -> c' that feed one output block.  The sign of a
// contribution is (-1)^{|M| n_l + |R_b| (n_l + n_c)} (graded tensor product).
#include "hpsi.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <unordered_map>

namespace bsd {

namespace {

struct LRef {
  int kind;      // 0 stored, 1 identity, 2 aggregate
  OpKey key;
  bool trans = false;
  int agg = -1;
  Q dq;
};

OpKey mk(char k, int p = -1, int q = -1) {
  OpKey o;
  o.kind = k;
  o.p = p;
  o.q = q;
  return o;
}

std::vector<Group> scale_groups(std::vector<Group> g, double c) {
  for (auto& x : g)
    for (auto& t : x.terms) t.coef *= c;
  return g;
}

}  // namespace

__global__ void zero_fill_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void zero_fill(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(grid), dim3(256), 0, s, p, n);
  BSD_HIP(hipGetLastError());
}

void build_psi_layout(const Block& Lb, const Block& Rb, const SiteSet& C, const Q& target,
                      PsiLayout& lay) {
  lay.blocks.clear();
  lay.stack_off.assign(Rb.basis.q.size(), -1);
  lay.stack_rows.assign(Rb.basis.q.size(), 0);
  lay.stack_prows.assign(Rb.basis.q.size(), 0);
  int64_t off = 0;
  for (int r = 0; r < (int)Rb.basis.q.size(); ++r) {
    int rows = 0, prows = 0;
    int64_t base = off;
    for (int l = 0; l < (int)Lb.basis.q.size(); ++l)
      for (int c = 0; c < 16; ++c) {
        if (Lb.basis.q[l] + C.q[c] + Rb.basis.q[r] != target) continue;
        PsiBlk b;
        b.l = l;
        b.c = c;
        b.r = r;
        b.rows = Lb.basis.dim[l];
        b.cols = Rb.basis.dim[r];
        b.off = off;
        b.row_in_stack = rows;
        b.prow_in_stack = prows;
        lay.index[{l, c, r}] = (int)lay.blocks.size();
        lay.blocks.push_back(b);
        off += (int64_t)b.rows * b.cols;
        rows += b.rows;
        prows += (b.rows + 7) / 8 * 8;
      }
    if (rows > 0) {
      lay.stack_off[r] = base;
      lay.stack_rows[r] = rows;
      lay.stack_prows[r] = prows;
    }
  }
  lay.n_elems = off;
}

static Operand2 lref_block(const Block& Lb, const LRef& r, const std::vector<Skeleton>& agg_sk,
                           const std::vector<int64_t>& agg_off, const double* agg_mem, int in_idx) {
  Operand2 o;
  const Basis& bs = Lb.basis;
  int out_idx = bs.find(bs.q[in_idx] + r.dq);
  if (out_idx < 0) return o;
  o.out = out_idx;
  if (r.kind == 1) {
    o.ident = true;
    o.ok = true;
    return o;
  }
  if (r.kind == 2) {
    int b = agg_sk[r.agg].by_in[in_idx];
    if (b < 0) return o;
    const SkBlock& sb = agg_sk[r.agg].blocks[b];
    o.p = agg_mem + agg_off[r.agg] + sb.off;
    o.ld = sb.ld;
    o.ok = true;
    return o;
  }
  int rr, cc, ld;
  const double* p = r.trans ? Lb.op_block(r.key, out_idx, &rr, &cc, &ld) : Lb.op_block(r.key, in_idx, &rr, &cc, &ld);
  if (!p) return o;
  o.p = p;
  o.ld = ld;
  o.trans = r.trans;
  o.ok = true;
  return o;
}

// pack of the streamed right operators: rows x ld float64 blocks gathered from
// the block's device memory into a contiguous buffer
__global__ void __launch_bounds__(256) gather_kernel(const StreamGather* __restrict__ g, double* __restrict__ dst) {
  const StreamGather t = g[blockIdx.x];
  for (int64_t e = threadIdx.x; e < t.n; e += blockDim.x) dst[t.off + e] = t.src[e];
}

// Slots and host packs of a streamed product: two device slots for the
// float64 operator packs and two for their planes (chunk k uses slot k % 2),
// the packs themselves in pinned host memory, filled here from the resident
// right block (gather on the device, one copy to the host per chunk).
void prepare_stream_slots(HpsiPlan& plan, std::vector<std::vector<GemmProblem>>& p1,
                          std::vector<std::vector<GemmProblem>>& p1s, std::vector<std::vector<GemmProblem>>& p1h,
                          hipStream_t s) {
  const int nchunks = (int)plan.schunks.size();
  int64_t smax = 32, pmax = 64;
  size_t host = 0;
  for (auto& sc : plan.schunks) {
    smax = std::max(smax, sc.elems);
    pmax = std::max(pmax, sc.pelems);
    sc.host_off = host;
    host += (size_t)sc.elems * sizeof(double);
  }
  plan.slot_bytes = (size_t)smax * sizeof(double);
  plan.pslot_bytes = (size_t)pmax * 2;
  plan.slots.reserve(2 * plan.slot_bytes);
  plan.pslots.reserve(2 * plan.pslot_bytes);
  BSD_HIP(hipHostMalloc(&plan.pack_host, std::max<size_t>(host, 256), hipHostMallocDefault));
  plan.pack_bytes = host;
  auto slot = [&](int k) { return static_cast<char*>(plan.slots.p) + (size_t)(k % 2) * plan.slot_bytes; };
  auto pslot = [&](int k) { return static_cast<char*>(plan.pslots.p) + (size_t)(k % 2) * plan.pslot_bytes; };
  auto fix = [&](uint64_t t, int k) -> uint64_t {
    const uint64_t tag = t >> kTagShift, off = t & ((1ull << kTagShift) - 1);
    if (tag == 4) return tag_ptr(0, (uint64_t)(uintptr_t)slot(k) + off);
    if (tag == 5) return tag_ptr(0, (uint64_t)(uintptr_t)pslot(k) + off);
    return t;
  };
  for (int k = 0; k < nchunks; ++k) {
    for (auto& gp : p1[k])
      for (auto& sg : gp.segs) sg.B = fix(sg.B, k);
    for (auto& gp : p1s[k])
      for (auto& sg : gp.segs) sg.B = fix(sg.B, k);
    for (auto& gp : p1h[k])
      for (auto& sg : gp.segs) sg.B = fix(sg.B, k);
    auto& sc = plan.schunks[k];
    for (auto& t : sc.split) {
      t.src = fix(t.src, k);
      t.dst = reinterpret_cast<uint16_t*>(pslot(k) + (uintptr_t)t.dst);
    }
    sc.split_dev.reserve(std::max<size_t>(1, sc.split.size()) * sizeof(SplitTask));
    if (!sc.split.empty())
      BSD_HIP(hipMemcpy(sc.split_dev.p, sc.split.data(), sc.split.size() * sizeof(SplitTask), hipMemcpyHostToDevice));
    // fill the pack: gather into slot 0, copy to the host
    if (!sc.gather.empty()) {
      DevBuf gl;
      gl.reserve(sc.gather.size() * sizeof(StreamGather));
      BSD_HIP(hipMemcpy(gl.p, sc.gather.data(), sc.gather.size() * sizeof(StreamGather), hipMemcpyHostToDevice));
      hipLaunchKernelGGL(gather_kernel, dim3((unsigned)sc.gather.size()), dim3(256), 0, s,
                         static_cast<const StreamGather*>(gl.p), reinterpret_cast<double*>(slot(0)));
      BSD_HIP(hipGetLastError());
      BSD_HIP(hipMemcpyAsync(static_cast<char*>(plan.pack_host) + sc.host_off, slot(0), (size_t)sc.elems * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      BSD_HIP(hipStreamSynchronize(s));
    }
    sc.gather.clear();
    sc.gather.shrink_to_fit();
    sc.where.clear();
  }
  BSD_HIP(hipStreamCreateWithFlags(&plan.side, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i) {
    BSD_HIP(hipEventCreateWithFlags(&plan.ev_loaded[i], hipEventDisableTiming));
    BSD_HIP(hipEventCreateWithFlags(&plan.ev_free[i], hipEventDisableTiming));
  }
}

std::unique_ptr<HpsiPlan> build_hpsi_plan(Ctx& ctx, int site, int precision, size_t ws_budget,
                                          hipStream_t s, bool stream_r) {
  Block* Lb = get_block(ctx, true, site);
  Block* Rb = get_block(ctx, false, site + 2);
  BSD_CHECK(Lb && Rb, 1, "environment blocks for this site are not built");
  BSD_CHECK(Lb->resident && Rb->resident, 6, "environment block is offloaded");
  // right operators per chunk: the set cap, or 1 GiB when streaming without one
  const int64_t kStreamChunkBytes =
      ctx.stream_chunk_bytes ? (int64_t)ctx.stream_chunk_bytes : (stream_r ? (int64_t)1 << 30 : 0);
  BSD_CHECK(!Rb->normal, 2, "the right block of this site holds normal operators; the product needs the "
                            "complementary set (build it with a smaller right_normal_from)");
  const SiteSet C = make_siteset(site, 2);
  const int nL = 2 * site;
  const int r0 = 2 * (site + 2), NM = 2 * ctx.L;
  auto plan = std::make_unique<HpsiPlan>();
  plan->site = site;
  plan->precision = precision;
  // BSDMRG_VERBOSE: host wall time of the stages
  const bool verbose = std::getenv("BSDMRG_VERBOSE") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  auto note = [&](const char* what) {
    if (!verbose) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "plan: %s %.3f s\n", what, std::chrono::duration<double>(now - t_last).count());
    t_last = now;
  };
  build_psi_layout(*Lb, *Rb, C, ctx.target, plan->lay);
  const PsiLayout& lay = plan->lay;

  // ---------------------------------------------------------------- channels
  struct Chan {
    int rkind;       // 0 stored, 1 identity
    OpKey rkey;
    bool rtrans = false;
    Q rdq;
    std::vector<Group> groups;
  };
  std::vector<Chan> chans;
  auto add = [&](int rkind, OpKey rkey, bool rtrans, std::vector<Group> g) {
    if (g.empty()) return;
    if (rkind == 0 && Rb->ops.find(rkey) == Rb->ops.end()) return;
    Chan c;
    c.rkind = rkind;
    c.rkey = rkey;
    c.rtrans = rtrans;
    Q dq = rkind == 1 ? Q{0, 0} : key_dq(rkey, false);
    c.rdq = rtrans ? -dq : dq;
    c.groups = std::move(g);
    chans.push_back(std::move(c));
  };
  const Mat I16 = mat_eye(16);
  add(1, mk('I'), false, expand_left(mk('H'), nL, C, ctx.ints));
  {
    Group g;
    g.M = I16;
    g.terms.push_back({1.0, mk('I'), false});
    add(0, mk('H'), false, {g});
  }
  for (int x = 0; x < r0; ++x) {
    auto g = expand_left(mk('c', x), nL, C, ctx.ints);
    add(0, mk('S', x), false, g);
    add(0, mk('S', x), true, scale_groups(transpose_groups(g, C, 1), -1.0));
  }
  for (int r = r0; r < NM; ++r) {
    auto g = expand_left(mk('S', r), nL, C, ctx.ints);
    add(0, mk('c', r), true, g);
    add(0, mk('c', r), false, scale_groups(transpose_groups(g, C, 1), -1.0));
  }
  for (int p = 0; p < r0; ++p)
    for (int q = p + 1; q < r0; ++q) {
      auto g = expand_left(mk('A', p, q), nL, C, ctx.ints);
      add(0, mk('P', p, q), false, g);
      add(0, mk('P', p, q), true, transpose_groups(g, C, 0));
    }
  for (int p = 0; p < r0; ++p)
    for (int q = 0; q < r0; ++q) add(0, mk('Q', p, q), false, expand_left(mk('B', p, q), nL, C, ctx.ints));

  // ---------------------------------------------------------------- L-side references
  std::vector<LRef> lrefs;
  std::map<std::tuple<int, char, int, int, bool>, int> lidx;
  std::vector<Skeleton> agg_sk;
  std::vector<int64_t> agg_off;
  std::vector<std::vector<Term>> agg_terms;
  int64_t agg_elems = 0;
  struct G2 {
    int lref;
    double coef;
    Mat M;
    int mpar;
  };
  std::vector<std::vector<G2>> cgroups(chans.size());
  for (size_t ci = 0; ci < chans.size(); ++ci) {
    Q total_dq = -chans[ci].rdq;
    for (auto& g : chans[ci].groups) {
      Q ldq;
      int mpar = -1;
      for (int a = 0; a < 16 && mpar < 0; ++a)
        for (int b = 0; b < 16; ++b)
          if (g.M(a, b) != 0.0) {
            ldq = C.q[a] - C.q[b];
            mpar = ldq.parity();
            break;
          }
      if (mpar < 0) continue;
      Q bdq = total_dq - ldq;
      std::vector<Term> kept;
      for (auto& t : g.terms) {
        if (t.key.kind != 'I' && Lb->ops.find(t.key) == Lb->ops.end()) continue;
        Q tdq = t.key.kind == 'I' ? Q{0, 0} : key_dq(t.key, true);
        if (t.trans) tdq = -tdq;
        BSD_CHECK(tdq == bdq, 1, "inconsistent dq in H.psi expansion");
        kept.push_back(t);
      }
      if (kept.empty()) continue;
      G2 g2;
      g2.M = g.M;
      g2.mpar = mpar;
      if (kept.size() == 1) {
        const Term& t = kept[0];
        int kind = t.key.kind == 'I' ? 1 : 0;
        auto id = std::make_tuple(kind, t.key.kind, t.key.p, t.key.q, t.trans);
        auto it = lidx.find(id);
        if (it == lidx.end()) {
          LRef r;
          r.kind = kind;
          r.key = t.key;
          r.trans = t.trans;
          r.dq = bdq;
          lidx[id] = (int)lrefs.size();
          g2.lref = (int)lrefs.size();
          lrefs.push_back(r);
        } else {
          g2.lref = it->second;
        }
        g2.coef = t.coef;
      } else {
        LRef r;
        r.kind = 2;
        r.agg = (int)agg_sk.size();
        r.dq = bdq;
        agg_sk.push_back(make_skeleton(Lb->basis, Lb->basis, bdq));
        agg_off.push_back(agg_elems);
        agg_elems += agg_sk.back().layer_stride;
        agg_terms.push_back(kept);
        g2.lref = (int)lrefs.size();
        lrefs.push_back(r);
        g2.coef = 1.0;
      }
      cgroups[ci].push_back(std::move(g2));
    }
  }
  plan->agg.reserve(std::max<int64_t>(1, agg_elems) * sizeof(double));
  double* agg_mem = static_cast<double*>(plan->agg.p);
  plan->agg_bytes = agg_elems * sizeof(double);
  {
    std::vector<AggTask> tasks;
    std::vector<AggTerm> terms;
    for (size_t a = 0; a < agg_sk.size(); ++a)
      for (const auto& sb : agg_sk[a].blocks) {
        AggTask t;
        t.out = agg_mem + agg_off[a] + sb.off;
        t.ldo = sb.ld;
        t.rows = sb.rows;
        t.cols = sb.cols;
        t.t0 = (int)terms.size();
        for (const auto& tm : agg_terms[a]) {
          AggTerm x;
          x.coef = tm.coef;
          x.pad = 0;
          if (tm.key.kind == 'I') {
            if (sb.in != sb.out) continue;
            x.in = nullptr;
            x.ldi = 0;
            x.flags = kIdentA;
          } else {
            int rr, cc, ld;
            const double* p = tm.trans ? Lb->op_block(tm.key, sb.out, &rr, &cc, &ld)
                                       : Lb->op_block(tm.key, sb.in, &rr, &cc, &ld);
            if (!p) continue;
            x.in = p;
            x.ldi = ld;
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
    if (!tasks.empty()) {
      DevBuf dt, dm;
      dt.reserve(tasks.size() * sizeof(AggTask));
      dm.reserve(std::max<size_t>(1, terms.size()) * sizeof(AggTerm));
      BSD_HIP(hipMemcpyAsync(dt.p, tasks.data(), tasks.size() * sizeof(AggTask), hipMemcpyHostToDevice, s));
      if (!terms.empty())
        BSD_HIP(hipMemcpyAsync(dm.p, terms.data(), terms.size() * sizeof(AggTerm), hipMemcpyHostToDevice, s));
      launch_aggregate((const AggTask*)dt.p, (const AggTerm*)dm.p, (int)tasks.size(), s);
      BSD_HIP(hipStreamSynchronize(s));
    }
  }

  note("channels and L-side references");
  // ---------------------------------------------------------------- chunks of channels
  const int nR = (int)Rb->basis.q.size();
  std::vector<std::vector<int>> by_c(16);
  for (int b = 0; b < (int)lay.blocks.size(); ++b) by_c[lay.blocks[b].c].push_back(b);
  // phase-1 V storage per channel: for each output right sector r' a stack rows x d_R(r')
  struct VInfo {
    std::vector<int64_t> off;   // per output right index, element offset in chunk workspace or -1
    std::vector<int> src;       // input right index feeding r'
    std::vector<int64_t> poff;  // per output right index, bf16 offset in the chunk's plane workspace
  };
  std::vector<VInfo> vinfo(chans.size());
  std::vector<int> chunk_of(chans.size());
  std::vector<int64_t> chunk_size, chunk_psize;
  int64_t cur = 0, curp = 0, curr = 0;
  // the workspace budget covers V (float64) and its split planes (bf16)
  const int64_t budget = (int64_t)ws_budget;
  for (size_t ci = 0; ci < chans.size(); ++ci) {
    auto& ch = chans[ci];
    VInfo vi;
    vi.off.assign(nR, -1);
    vi.src.assign(nR, -1);
    vi.poff.assign(nR, -1);
    int64_t need = 0, needp = 0, needr = 0;
    if (ch.rkind == 0) {
      for (int r = 0; r < nR; ++r) {
        if (lay.stack_rows[r] == 0) continue;
        int r2 = Rb->basis.find(Rb->basis.q[r] + ch.rdq);
        if (r2 < 0) continue;
        int rr, cc, ld;
        const double* p = ch.rtrans ? Rb->op_block(ch.rkey, r2, &rr, &cc, &ld) : Rb->op_block(ch.rkey, r, &rr, &cc, &ld);
        if (!p) continue;
        vi.off[r2] = need;   // relative, fixed below
        vi.poff[r2] = needp;
        vi.src[r2] = r;
        need += ((int64_t)lay.stack_rows[r] * Rb->basis.dim[r2] + 1) / 2 * 2;
        needp += plane_elems(Rb->basis.dim[r2], lay.stack_prows[r] / 8);
        needr += (int64_t)rr * ld;
      }
      if (need == 0) {
        cgroups[ci].clear();
        chunk_of[ci] = -1;
        vinfo[ci] = vi;
        continue;
      }
    }
    const auto bytes = [](int64_t v, int64_t pl) { return v * (int64_t)sizeof(double) + pl * 2; };
    // streamed right operators: a chunk also holds at most kStreamChunkBytes of them
    const bool rfull = kStreamChunkBytes > 0 && curr > 0 && (curr + needr) * (int64_t)sizeof(double) > kStreamChunkBytes;
    if (chunk_size.empty() || rfull || (bytes(cur + need, curp + needp) > budget && (cur > 0 || curp > 0))) {
      chunk_size.push_back(0);
      chunk_psize.push_back(0);
      cur = 0;
      curp = 0;
      curr = 0;
    }
    curr += needr;
    for (auto& o : vi.off)
      if (o >= 0) o += cur;
    for (auto& o : vi.poff)
      if (o >= 0) o += curp;
    cur += need;
    curp += needp;
    chunk_size.back() = cur;
    chunk_psize.back() = curp;
    chunk_of[ci] = (int)chunk_size.size() - 1;
    vinfo[ci] = vi;
  }
  int64_t ws_elems = 0, vp_elems = 0;
  for (auto c : chunk_size) ws_elems = std::max(ws_elems, c);
  for (auto c : chunk_psize) vp_elems = std::max(vp_elems, c);
  plan->V.reserve(std::max<int64_t>(1, ws_elems) * sizeof(double));
  plan->v_bytes = ws_elems * sizeof(double);

  // plane arena (bf16 elements): [V planes of one chunk | psi planes | L-operator planes]
  const int64_t psip_base = vp_elems;
  std::vector<int64_t> psi_poff(lay.blocks.size());
  int64_t arena = psip_base;
  for (size_t bi = 0; bi < lay.blocks.size(); ++bi) {
    const PsiBlk& pb = lay.blocks[bi];
    psi_poff[bi] = arena;
    arena += plane_elems(pb.cols, (pb.rows + 7) / 8);
  }
  // psi row planes per right-sector stack, rows padded to the 8-row block starts
  std::vector<int64_t> psir_off(nR, -1);
  for (int r = 0; r < nR; ++r) {
    if (lay.stack_rows[r] == 0) continue;
    psir_off[r] = arena;
    arena += plane_elems(lay.stack_prows[r], (Rb->basis.dim[r] + 7) / 8);
  }
  // operator planes (left and right blocks), split once when the plan is built
  std::map<std::pair<const double*, bool>, int64_t> op_planes;   // (block, transposed) -> arena offset
  std::vector<SplitTask> op_tasks;
  auto op_plane = [&](const double* p, int64_t ld, bool trans, int rows, int K) -> int64_t {
    auto key = std::make_pair(p, trans);
    auto it = op_planes.find(key);
    if (it != op_planes.end()) return it->second;
    SplitTask t;
    t.src = tag_ptr(0, (uint64_t)p);
    t.lds = ld;
    t.kmap = nullptr;
    t.rmap = nullptr;
    t.dst = reinterpret_cast<uint16_t*>((uintptr_t)(arena * 2));   // arena byte offset, fixed below
    t.rows = rows;
    t.kcols = K;
    t.chunks = (K + 7) / 8;
    t.trans = trans ? 1 : 0;
    op_tasks.push_back(t);
    op_planes[key] = arena;
    const int64_t at = arena;
    arena += plane_elems(rows, t.chunks);
    return at;
  };
  double* V = static_cast<double*>(plan->V.p);
  const int nchunks = (int)chunk_size.size();
  plan->phase1.resize(nchunks);
  plan->phase2.resize(nchunks);
  double useful = 0.0;

  plan->stream_r = stream_r;
  if (stream_r) plan->schunks.resize(nchunks);
  // distinct operator blocks the product reads (algorithmic bytes: each once)
  std::unordered_map<const double*, int64_t> op_blocks;
  double heavy_flops = 0.0, ident_flops = 0.0;   // diagnostics
  std::vector<std::vector<GemmProblem>> p1(nchunks), p1s(nchunks), p1h(nchunks);
  // per chunk, per output psi block: list of segments
  // (dense by output psi block; empty entries are skipped when the lists are handed on)
  const int nblk = (int)lay.blocks.size();
  std::vector<std::vector<GemmProblem>> p2(nchunks), p2s(nchunks), p2h(nchunks);
  for (int k = 0; k < nchunks; ++k) {
    p2[k].resize(nblk);
    p2s[k].resize(nblk);
    p2h[k].resize(nblk);
  }
  // psi block of (left index, local state, right index), dense
  const int nLs = (int)Lb->basis.q.size(), nRs = (int)Rb->basis.q.size();
  std::vector<int> bidx((size_t)nLs * 16 * nRs, -1);
  for (int b = 0; b < nblk; ++b)
    bidx[((size_t)lay.blocks[b].l * 16 + lay.blocks[b].c) * nRs + lay.blocks[b].r] = b;
  for (size_t ci = 0; ci < chans.size(); ++ci) {
    if (chunk_of[ci] < 0 || cgroups[ci].empty()) continue;
    const int ck = chunk_of[ci];
    const auto& ch = chans[ci];
    const auto& vi = vinfo[ci];
    // the channels with the largest operators (the block Hamiltonians and the
    // diagonal two-index terms, which carry the particle-number-dependent bulk
    // of the energy) run in float64 on the split path too
    const bool heavy = ctx.heavy_fp64 && (ch.rkind == 1 || ch.rkey.kind == 'H' ||
                                          (ch.rkey.kind == 'Q' && ch.rkey.p == ch.rkey.q));
    if (ch.rkind == 0) {
      for (int r2 = 0; r2 < nR; ++r2) {
        if (vi.off[r2] < 0) continue;
        int r = vi.src[r2];
        int rr, cc, ld;
        const double* p = ch.rtrans ? Rb->op_block(ch.rkey, r2, &rr, &cc, &ld) : Rb->op_block(ch.rkey, r, &rr, &cc, &ld);
        op_blocks[p] = (int64_t)rr * cc;
        // streamed: the block sits in chunk ck's pack (rows x ld float64 at roff),
        // its planes in the chunk's plane slot (at rpoff), both resolved below
        int64_t roff = -1, rpoff = -1;
        if (stream_r) {
          auto& sc = plan->schunks[ck];
          auto it = sc.where.find(std::make_pair(p, ch.rtrans));
          if (it == sc.where.end()) {
            roff = sc.elems;
            sc.elems += ((int64_t)rr * ld + 31) / 32 * 32;
            rpoff = sc.pelems;
            sc.pelems += plane_elems(Rb->basis.dim[r2], (Rb->basis.dim[r] + 7) / 8);
            sc.where[std::make_pair(p, ch.rtrans)] = std::make_pair(roff, rpoff);
            sc.gather.push_back({p, roff, (int64_t)rr * ld});
            SplitTask t;
            t.src = tag_ptr(4, (uint64_t)(roff * sizeof(double)));
            t.lds = ld;
            t.kmap = nullptr;
            t.rmap = nullptr;
            t.dst = reinterpret_cast<uint16_t*>((uintptr_t)(rpoff * 2));
            t.rows = Rb->basis.dim[r2];
            t.kcols = Rb->basis.dim[r];
            t.chunks = (Rb->basis.dim[r] + 7) / 8;
            t.trans = ch.rtrans ? 1 : 0;
            sc.split.push_back(t);
          } else {
            roff = it->second.first;
            rpoff = it->second.second;
          }
        }
        GemmProblem gp;
        gp.C = tag_ptr(0, (uint64_t)(V + vi.off[r2]));
        gp.ldc = Rb->basis.dim[r2];
        gp.M = lay.stack_rows[r];
        gp.N = Rb->basis.dim[r2];
        gp.beta = 0.0;
        GSeg sg;
        sg.A = tag_ptr(1, (uint64_t)(lay.stack_off[r] * sizeof(double)));
        sg.lda = Rb->basis.dim[r];
        sg.B = stream_r ? tag_ptr(4, (uint64_t)(roff * sizeof(double))) : tag_ptr(0, (uint64_t)p);
        sg.ldb = ld;
        sg.K = Rb->basis.dim[r];
        sg.flags = ch.rtrans ? 0 : kTransB;   // op(B) = R_b^T
        sg.alpha = 1.0;
        gp.segs.push_back(sg);
        useful += 2.0 * gp.M * (double)gp.N * sg.K;
        if (heavy) heavy_flops += 2.0 * gp.M * (double)gp.N * sg.K;
        if (heavy) p1h[ck].push_back(gp);
        p1[ck].push_back(std::move(gp));
        if (heavy) continue;
        // split precision: psi row planes times planes of R_b, stored as the
        // planes of V^T (rows r', K = padded stack rows) that phase 2 reads
        GemmProblem gs;
        gs.C = tag_ptr(3, (uint64_t)(vi.poff[r2] * 2));
        gs.ldc = lay.stack_prows[r] / 8;
        gs.M = lay.stack_prows[r];
        gs.N = Rb->basis.dim[r2];
        gs.beta = 0.0;
        GSeg sq;
        sq.A = tag_ptr(3, (uint64_t)(psir_off[r] * 2));
        sq.lda = (Rb->basis.dim[r] + 7) / 8;
        sq.B = stream_r ? tag_ptr(5, (uint64_t)(rpoff * 2))
                        : tag_ptr(3, (uint64_t)(op_plane(p, ld, ch.rtrans, Rb->basis.dim[r2], Rb->basis.dim[r]) * 2));
        sq.ldb = (Rb->basis.dim[r] + 7) / 8;
        sq.K = Rb->basis.dim[r];
        sq.flags = 0;
        sq.alpha = 1.0;
        gs.segs.push_back(sq);
        p1s[ck].push_back(std::move(gs));
      }
    }
    const int rpar = ch.rdq.parity();
    // what an input block contributes does not depend on the output local
    // state c2: its right sector, L operand and plane offset are found once per
    // (group, c) and reused for every c2 (the segment order is unchanged)
    struct InBlk {
      int r2 = -1;
      Operand2 o;
      int64_t plane = -1;   // op_plane of o, taken at its first use
    };
    std::vector<InBlk> inb;
    for (const auto& g : cgroups[ci]) {
      const LRef& lr = lrefs[g.lref];
      for (int c = 0; c < 16; ++c) {
        bool any = false;
        for (int c2 = 0; c2 < 16 && !any; ++c2) any = g.M(c2, c) != 0.0;
        if (!any) continue;
        inb.assign(by_c[c].size(), InBlk());
        for (size_t k = 0; k < by_c[c].size(); ++k) {
          const PsiBlk& pb = lay.blocks[by_c[c][k]];
          int r2 = ch.rkind == 1 ? pb.r : Rb->basis.find(Rb->basis.q[pb.r] + ch.rdq);
          if (r2 < 0) continue;
          if (ch.rkind == 0 && (vi.off[r2] < 0 || vi.src[r2] != pb.r)) continue;
          Operand2 o = lref_block(*Lb, lr, agg_sk, agg_off, agg_mem, pb.l);
          if (!o.ok) continue;
          inb[k].r2 = r2;
          inb[k].o = o;
        }
        for (int c2 = 0; c2 < 16; ++c2) {
          double m = g.M(c2, c);
          if (m == 0.0) continue;
          for (size_t k = 0; k < by_c[c].size(); ++k) {
            InBlk& ib = inb[k];
            if (ib.r2 < 0) continue;
            const int bi = by_c[c][k];
            const PsiBlk& pb = lay.blocks[bi];
            // input block (l, c, r); output (l', c2, r')
            const int r2 = ib.r2;
            const Operand2& o = ib.o;
            const int oidx = bidx[((size_t)o.out * 16 + c2) * nRs + r2];
            if (oidx < 0) continue;
            const PsiBlk& ob = lay.blocks[oidx];
            const int lpar = Lb->basis.q[pb.l].parity();
            const int cpar = C.q[c].parity();
            int sp = (g.mpar & lpar) ^ (rpar & (lpar ^ cpar));
            GSeg sg;
            sg.alpha = g.coef * m * (sp ? -1.0 : 1.0);
            sg.K = pb.rows;
            sg.flags = (o.trans ? kTransA : 0) | (o.ident ? kIdentA : 0);
            sg.A = tag_ptr(0, (uint64_t)o.p);
            sg.lda = o.ld;
            if (ch.rkind == 1) {
              sg.B = tag_ptr(1, (uint64_t)(pb.off * sizeof(double)));
              sg.ldb = pb.cols;
            } else {
              int64_t row0 = pb.row_in_stack;
              sg.B = tag_ptr(0, (uint64_t)(V + vi.off[r2] + row0 * Rb->basis.dim[r2]));
              sg.ldb = Rb->basis.dim[r2];
            }
            auto& gp = p2[ck][oidx];
            if (gp.segs.empty()) {
              gp.C = tag_ptr(2, (uint64_t)(ob.off * sizeof(double)));
              gp.ldc = ob.cols;
              gp.M = ob.rows;
              gp.N = ob.cols;
              gp.beta = 1.0;
              gp.group = ob.r;   // outputs of one right sector read the same V_b columns
            }
            gp.segs.push_back(sg);
            if (!o.ident) {
              useful += 2.0 * ob.rows * (double)ob.cols * pb.rows;
              op_blocks[o.p] = (int64_t)ob.rows * pb.rows;
              if (heavy) heavy_flops += 2.0 * ob.rows * (double)ob.cols * pb.rows;
              if (ch.rkind == 1) ident_flops += 2.0 * ob.rows * (double)ob.cols * pb.rows;
            }
            if (heavy) {
              auto& gh = p2h[ck][oidx];
              if (gh.segs.empty()) {
                gh.C = gp.C;
                gh.ldc = gp.ldc;
                gh.M = gp.M;
                gh.N = gp.N;
                gh.beta = 1.0;
                gh.group = gp.group;
              }
              gh.segs.push_back(sg);
              continue;
            }
            // the same product on split planes: A rows of op(Lambda), B rows of V^T (or psi^T)
            GSeg sq;
            sq.alpha = sg.alpha;
            sq.K = pb.rows;
            sq.flags = o.ident ? kIdentA : 0;
            if (!o.ident && ib.plane < 0) ib.plane = op_plane(o.p, o.ld, o.trans, ob.rows, pb.rows);
            sq.A = o.ident ? tag_ptr(3, 0) : tag_ptr(3, (uint64_t)(ib.plane * 2));
            sq.lda = (pb.rows + 7) / 8;
            if (ch.rkind == 1) {
              sq.B = tag_ptr(3, (uint64_t)(psi_poff[bi] * 2));
              sq.ldb = (pb.rows + 7) / 8;
            } else {
              const int64_t e = vi.poff[r2] + plane_off(0, pb.prow_in_stack / 8, 0, lay.stack_prows[pb.r] / 8);
              sq.B = tag_ptr(3, (uint64_t)(e * 2));
              sq.ldb = lay.stack_prows[pb.r] / 8;
            }
            auto& gq = p2s[ck][oidx];
            if (gq.segs.empty()) {
              gq.C = gp.C;
              gq.ldc = gp.ldc;
              gq.M = gp.M;
              gq.N = gp.N;
              gq.beta = 1.0;
              gq.group = gp.group;
            }
            gq.segs.push_back(sq);
          }
        }
      }
    }
  }
  note("segments");
  // diagonal of H_eff: for every channel and group without a quantum-number
  // change, diag(Lambda) (x) M[c][c] (x) diag(R_b), as K = 1 sector products
  {
    int maxd = 1;
    for (int d : Lb->basis.dim) maxd = std::max(maxd, d);
    for (int d : Rb->basis.dim) maxd = std::max(maxd, d);
    plan->ones.reserve(maxd * sizeof(double));
    std::vector<double> ones(maxd, 1.0);
    BSD_HIP(hipMemcpy(plan->ones.p, ones.data(), maxd * sizeof(double), hipMemcpyHostToDevice));
    const double* one = static_cast<const double*>(plan->ones.p);
    std::map<int, GemmProblem> dprob;
    for (size_t ci = 0; ci < chans.size(); ++ci) {
      const auto& ch = chans[ci];
      if (ch.rdq != Q{0, 0}) continue;
      for (const auto& g : cgroups[ci]) {
        const LRef& lr = lrefs[g.lref];
        if (lr.dq != Q{0, 0}) continue;
        for (int c = 0; c < 16; ++c) {
          const double m = g.M(c, c);
          if (m == 0.0) continue;
          for (int bi : by_c[c]) {
            const PsiBlk& pb = lay.blocks[bi];
            Operand2 o = lref_block(*Lb, lr, agg_sk, agg_off, agg_mem, pb.l);
            if (!o.ok) continue;
            GSeg sg;
            sg.K = 1;
            sg.alpha = g.coef * m;
            sg.A = tag_ptr(0, (uint64_t)(o.ident ? one : o.p));
            sg.lda = o.ident ? 1 : o.ld + 1;
            if (ch.rkind == 1) {
              sg.B = tag_ptr(0, (uint64_t)one);
              sg.ldb = 1;
            } else {
              int rr, cc, ld;
              const double* p = Rb->op_block(ch.rkey, pb.r, &rr, &cc, &ld);
              if (!p) continue;
              sg.B = tag_ptr(0, (uint64_t)p);
              sg.ldb = ld + 1;
            }
            sg.flags = kTransB;
            auto& gp = dprob[bi];
            if (gp.segs.empty()) {
              gp.C = tag_ptr(2, (uint64_t)(pb.off * sizeof(double)));
              gp.ldc = pb.cols;
              gp.M = pb.rows;
              gp.N = pb.cols;
              gp.beta = 1.0;
            }
            gp.segs.push_back(sg);
          }
        }
      }
    }
    std::vector<GemmProblem> v;
    for (auto& kv : dprob) v.push_back(std::move(kv.second));
    plan->diag_plan = std::make_unique<GemmPlan>();
    plan->diag_plan->build(v, true);
  }
  // plane arena: allocate now and turn arena offsets (tag 3) into absolute
  // addresses, which the plane kernels read through buffer descriptors
  plan->plane_bytes = (size_t)arena * 2;
  plan->planes.reserve(std::max<size_t>(16, plan->plane_bytes));
  const uint64_t arena_base = (uint64_t)(uintptr_t)plan->planes.p;
  auto absolute = [&](uint64_t t) {
    return (t >> kTagShift) == 3 ? tag_ptr(0, arena_base + (t & ((1ull << kTagShift) - 1))) : t;
  };
  for (int k = 0; k < nchunks; ++k) {
    for (auto& gp : p1s[k]) {
      gp.C = absolute(gp.C);
      for (auto& sg : gp.segs) {
        sg.A = absolute(sg.A);
        sg.B = absolute(sg.B);
      }
    }
    for (auto& gp : p2s[k])
      for (auto& sg : gp.segs) {
        sg.A = absolute(sg.A);
        sg.B = absolute(sg.B);
      }
  }
  if (stream_r) prepare_stream_slots(*plan, p1, p1s, p1h, s);
  plan->nseg = 0;
  plan->phase1s.resize(nchunks);
  plan->phase2s.resize(nchunks);
  plan->p2_probs.resize(nchunks);
  plan->p2s_probs.resize(nchunks);
  plan->p2h_probs.resize(nchunks);
  plan->phase1h.resize(nchunks);
  plan->phase2h.resize(nchunks);
  for (int k = 0; k < nchunks; ++k) {
    plan->phase1[k] = std::make_unique<GemmPlan>();
    plan->phase1s[k] = std::make_unique<GemmPlan>();
    plan->phase1h[k] = std::make_unique<GemmPlan>();
  }
  parallel_jobs(3 * nchunks, [&](int j, hipStream_t up) {
    const int k = j / 3;
    GemmBuildOpts o;
    o.upload = up;
    if (j % 3 == 0) {
      plan->phase1[k]->build(p1[k], o);
    } else if (j % 3 == 1) {
      o.plane_output = true;
      o.wave_max = 32;   // blocks above 32 x 32: 64 x 64 workgroup tiles
      plan->phase1s[k]->build(p1s[k], o);
    } else {
      plan->phase1h[k]->build(p1h[k], o);
    }
  });
  for (int k = 0; k < nchunks; ++k) {
    for (auto& gp : p2[k]) {
      if (gp.segs.empty()) continue;
      plan->nseg += gp.segs.size();
      plan->p2_probs[k].push_back(std::move(gp));
    }
    for (auto& gp : p2s[k])
      if (!gp.segs.empty()) plan->p2s_probs[k].push_back(std::move(gp));
    for (auto& gp : p2h[k])
      if (!gp.segs.empty()) plan->p2h_probs[k].push_back(std::move(gp));
  }
  if (std::getenv("BSDMRG_PLAN_STATS")) {
    // diagnostic: MFMA work of phase 2 at the kernels' granularity (16 x 16
    // tiles, K in passes of 32 values) against K padded to single chunks of 8
    // values, and how many K-segments carry |alpha| = 1
    double useful2 = 0, pad32 = 0, pad8 = 0, nseg2 = 0, unit = 0, nprob = 0, runs = 0, distinct = 0;
    for (const auto& v : plan->p2s_probs)
      for (const auto& gp : v) {
        nprob += 1;
        const double mp = (gp.M + 15) / 16 * 16.0, np_ = (gp.N + 15) / 16 * 16.0;
        double prev = 0;
        std::vector<double> mags;
        for (const auto& sg : gp.segs) mags.push_back(std::fabs(sg.alpha));
        std::sort(mags.begin(), mags.end());
        distinct += (double)(std::unique(mags.begin(), mags.end()) - mags.begin());
        for (const auto& sg : gp.segs) {
          nseg2 += 1;
          if (sg.flags & kIdentA) continue;
          useful2 += (double)gp.M * gp.N * sg.K;
          pad32 += mp * np_ * ((sg.K + 31) / 32 * 32.0);
          pad8 += mp * np_ * ((sg.K + 7) / 8 * 8.0);
          if (std::fabs(std::fabs(sg.alpha) - 1.0) == 0.0) unit += 1;
          if (std::fabs(sg.alpha) != prev) runs += 1;
          prev = std::fabs(sg.alpha);
        }
      }
    std::fprintf(stderr, "plan stats: useful flops %.3e, float64-policy channels %.1f%%, identity channel %.1f%%\n",
                 useful, 100.0 * heavy_flops / std::max(1.0, useful), 100.0 * ident_flops / std::max(1.0, useful));
    std::fprintf(stderr,
                 "plan stats: phase-2 problems %.0f, segments %.0f, |alpha|=1 %.1f%%, |alpha| runs %.0f, distinct "
                 "|alpha| per problem %.1f; MFMA work / useful: K by 32 %.3f, K by 8 %.3f\n",
                 nprob, nseg2, 100.0 * unit / std::max(1.0, nseg2), runs, distinct / std::max(1.0, nprob),
                 pad32 / std::max(1.0, useful2),
                 pad8 / std::max(1.0, useful2));
  }
  // phase-2 tile lists from the kept problem lists (the autotuner rebuilds
  // them); default schedule: wave tiles for every block and a split-K target
  // that grows with the number of K-segments (one wave per ~128 segments,
  // 8192 to 131072 waves): small products lose more to the part reduction
  // than they gain in parallelism, large ones the reverse
  plan->opts64.wave_max = 1 << 30;
  plan->opts_planes.wave_max = 32;   // blocks above 32 x 32: 64 x 64 workgroup tiles
  plan->opts64.target_waves = plan->opts_planes.target_waves =
      std::min(131072.0, std::max(8192.0, (double)plan->nseg / 128.0));
  rebuild_phase2(*plan, plan->opts64, plan->opts_planes, 3);

  note("diagonal, phase-1 lists and phase-2 tile lists");
  // ---------------------------------------------------------------- split tasks
  // padded-row maps of the right-sector stacks: plane column -> stack row or -1
  std::vector<int64_t> kmap_off(nR, -1);
  std::vector<int32_t> kmap;
  for (int r = 0; r < nR; ++r) {
    if (lay.stack_rows[r] == 0) continue;
    kmap_off[r] = (int64_t)kmap.size();
    kmap.resize(kmap.size() + lay.stack_prows[r], -1);
  }
  for (const auto& pb : lay.blocks)
    for (int i = 0; i < pb.rows; ++i) kmap[kmap_off[pb.r] + pb.prow_in_stack + i] = pb.row_in_stack + i;
  plan->kmaps.reserve(std::max<size_t>(1, kmap.size()) * sizeof(int32_t));
  if (!kmap.empty())
    BSD_HIP(hipMemcpy(plan->kmaps.p, kmap.data(), kmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  const int32_t* kmap_dev = static_cast<const int32_t*>(plan->kmaps.p);
  uint16_t* ar = static_cast<uint16_t*>(plan->planes.p);
  std::vector<SplitTask> tasks;
  for (size_t bi = 0; bi < lay.blocks.size(); ++bi) {
    const PsiBlk& pb = lay.blocks[bi];
    SplitTask t;
    t.src = tag_ptr(1, (uint64_t)(pb.off * sizeof(double)));
    t.lds = pb.cols;
    t.kmap = nullptr;
    t.rmap = nullptr;
    t.dst = ar + psi_poff[bi];
    t.rows = pb.cols;
    t.kcols = pb.rows;
    t.chunks = (pb.rows + 7) / 8;
    t.trans = 1;
    tasks.push_back(t);
  }
  for (int r = 0; r < nR; ++r) {
    if (lay.stack_rows[r] == 0) continue;
    SplitTask t;
    t.src = tag_ptr(1, (uint64_t)(lay.stack_off[r] * sizeof(double)));
    t.lds = Rb->basis.dim[r];
    t.kmap = nullptr;
    t.rmap = kmap_dev + kmap_off[r];
    t.dst = ar + psir_off[r];
    t.rows = lay.stack_prows[r];
    t.kcols = Rb->basis.dim[r];
    t.chunks = (Rb->basis.dim[r] + 7) / 8;
    t.trans = 0;
    tasks.push_back(t);
  }
  plan->n_split_psi = (int)tasks.size();
  plan->split_tasks.reserve(std::max<size_t>(1, tasks.size()) * sizeof(SplitTask));
  if (!tasks.empty())
    BSD_HIP(hipMemcpy(plan->split_tasks.p, tasks.data(), tasks.size() * sizeof(SplitTask), hipMemcpyHostToDevice));
  // operator planes: split once here
  if (!op_tasks.empty()) {
    for (auto& t : op_tasks) t.dst = ar + (int64_t)((uintptr_t)t.dst / 2);
    DevBuf dt;
    dt.reserve(op_tasks.size() * sizeof(SplitTask));
    BSD_HIP(hipMemcpyAsync(dt.p, op_tasks.data(), op_tasks.size() * sizeof(SplitTask), hipMemcpyHostToDevice, s));
    GBases b0{{0, 0, 0, 0}};
    launch_split_planes(static_cast<const SplitTask*>(dt.p), (int)op_tasks.size(), b0, s);
    BSD_HIP(hipStreamSynchronize(s));
  }
  plan->useful_flops = useful;
  plan->op_elems = 0;
  for (const auto& kv : op_blocks) plan->op_elems += kv.second;
  plan->nchannels = (int)chans.size();
  plan->naggs = (int)agg_sk.size();
  note("split tasks");
  return plan;
}

void rebuild_phase2(HpsiPlan& plan, const GemmBuildOpts& o64, const GemmBuildOpts& oplanes, int which) {
  const int nchunks = (int)plan.p2_probs.size();
  for (auto& g : plan.graphs) (void)hipGraphExecDestroy(g.exec);
  plan.graphs.clear();
  plan.opts64 = o64;
  plan.opts_planes = oplanes;
  plan.opts_planes.plane_operands = true;
  plan.opts64.upload = plan.opts_planes.upload = nullptr;
  plan.phase2h.resize(nchunks);
  for (int k = 0; k < nchunks; ++k) {
    if (which & 1) plan.phase2[k] = std::make_unique<GemmPlan>();
    if (which & 2) plan.phase2s[k] = std::make_unique<GemmPlan>();
    plan.phase2h[k] = std::make_unique<GemmPlan>();
  }
  parallel_jobs(3 * nchunks, [&](int j, hipStream_t up) {
    const int k = j / 3;
    if (j % 3 == 2) {
      // float64 channels of the split path follow the float64 schedule
      GemmBuildOpts o = plan.opts64;
      o.upload = up;
      plan.phase2h[k]->build(plan.p2h_probs[k], o);
    } else if (j % 3 == 0 && (which & 1)) {
      GemmBuildOpts o = plan.opts64;
      o.upload = up;
      plan.phase2[k]->build(plan.p2_probs[k], o);
    } else if (j % 3 == 1 && (which & 2)) {
      GemmBuildOpts o = plan.opts_planes;
      o.upload = up;
      plan.phase2s[k]->build(plan.p2s_probs[k], o);
    }
  });
}

TuneResult autotune_hpsi(HpsiPlan& plan, int precision, hipStream_t s) {
  const int64_t n = plan.lay.n_elems;
  DevBuf x, y;
  x.reserve(std::max<int64_t>(1, n) * sizeof(double));
  y.reserve(std::max<int64_t>(1, n) * sizeof(double));
  {
    // any fixed non-trivial vector will do: the schedule does not depend on values
    std::vector<double> h(std::max<int64_t>(1, n));
    uint64_t z = 0x9E3779B97F4A7C15ull;
    for (auto& v : h) {
      z ^= z << 13;
      z ^= z >> 7;
      z ^= z << 17;
      v = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    BSD_HIP(hipMemcpy(x.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  const double* xp = static_cast<const double*>(x.p);
  double* yp = static_cast<double*>(y.p);
  // candidate schedules
  std::vector<std::pair<GemmBuildOpts, GemmBuildOpts>> cand;
  const GemmBuildOpts base64 = plan.opts64, basep = plan.opts_planes;
  cand.push_back({base64, basep});
  for (double tw : {4096.0, 8192.0, 16384.0, 32768.0, 65536.0, 131072.0})
    for (int xcd = 0; xcd < 2; ++xcd)
      for (int wm : {32, 64, 128, 1 << 30}) {
        GemmBuildOpts a = base64, b = basep;
        if (precision == 0) {
          a.target_waves = tw;
          a.xcd_order = xcd;
          a.wave_max = wm;
        } else {
          if (wm != 32 && wm != (1 << 30)) continue;   // workgroup tiles above 32, or wave tiles only
          b.target_waves = tw;
          b.xcd_order = xcd;
          b.wave_max = wm;
        }
        cand.push_back({a, b});
      }
  const int which = precision == 0 ? 1 : 2;
  hipEvent_t e0, e1;
  BSD_HIP(hipEventCreate(&e0));
  BSD_HIP(hipEventCreate(&e1));
  auto time_it = [&]() {
    run_hpsi_graph(plan, xp, yp, s, precision);   // capture + warm-up
    BSD_HIP(hipStreamSynchronize(s));
    float best = 1e30f;
    for (int r = 0; r < 5; ++r) {
      BSD_HIP(hipEventRecord(e0, s));
      run_hpsi_graph(plan, xp, yp, s, precision);
      BSD_HIP(hipEventRecord(e1, s));
      BSD_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      BSD_HIP(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, ms);
    }
    return (double)best;
  };
  TuneResult res;
  res.n_candidates = (int)cand.size();
  double best = 1e300;
  const bool verbose = std::getenv("BSDMRG_VERBOSE") != nullptr;
  for (size_t i = 0; i < cand.size(); ++i) {
    rebuild_phase2(plan, cand[i].first, cand[i].second, which);
    const double ms = time_it();
    if (verbose) {
      const GemmBuildOpts& o = precision == 0 ? cand[i].first : cand[i].second;
      std::fprintf(stderr, "autotune: candidate %zu/%zu (waves %.0f, xcd %d, wave_max %d): %.3f ms\n", i + 1,
                   cand.size(), o.target_waves, (int)o.xcd_order, o.wave_max, ms);
    }
    if (i == 0) res.default_ms = ms;
    if (ms < best) {
      best = ms;
      res.best = (int)i;
    }
  }
  rebuild_phase2(plan, cand[res.best].first, cand[res.best].second, which);
  res.best_ms = best;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

static GBases hpsi_bases(const HpsiPlan& plan, const double* psi, double* out) {
  return GBases{{0, (uint64_t)psi, (uint64_t)out, (uint64_t)plan.planes.p}};
}

int profile_hpsi(const HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision, int cap,
                 double* ms, double* flops, double* bytes, int* kind) {
  // kind: 0 zero-fill, 1 split of psi into bf16 planes, 10 + c phase-1 grouped GEMM with tile shape class c, 20 + c phase 2,
  // 10 + kShapes / 20 + kShapes the split-K reduction of phase 1 / phase 2
  std::vector<hipEvent_t> ev;
  std::vector<int> kinds;
  std::vector<double> fl, by;
  auto mark = [&]() {
    hipEvent_t e;
    BSD_HIP(hipEventCreate(&e));
    BSD_HIP(hipEventRecord(e, s));
    ev.push_back(e);
  };
  const GBases b = hpsi_bases(plan, psi, out);
  const SplitTask* tasks = static_cast<const SplitTask*>(plan.split_tasks.p);
  mark();
  zero_fill(out, plan.lay.n_elems, s);
  kinds.push_back(0);
  fl.push_back(0.0);
  by.push_back(8.0 * plan.lay.n_elems);
  mark();
  if (precision != 0 && plan.n_split_psi > 0) {
    launch_split_planes(tasks, plan.n_split_psi, b, s);
    kinds.push_back(1);
    fl.push_back(0.0);
    by.push_back(plan.lay.n_elems * (8.0 + 2.0 * 2 * kPlaneParts));   // psi read, two plane copies written
    mark();
  }
  for (size_t k = 0; k < plan.phase1.size(); ++k) {
    // split precision: the float64 channels first (kinds 30 + c, 40 + c)
    for (int ph = (precision == 0 ? 1 : -2); ph <= 2; ++ph) {
      if (ph == 0) continue;
      const bool h = ph < 0;
      const int phase = h ? ph + 3 : ph;
      const GemmPlan& gp = h ? (phase == 1 ? *plan.phase1h[k] : *plan.phase2h[k])
                             : precision == 0 ? (phase == 1 ? *plan.phase1[k] : *plan.phase2[k])
                                              : (phase == 1 ? *plan.phase1s[k] : *plan.phase2s[k]);
      const int prec = h ? 0 : precision;
      const int base = (h ? 20 : 0) + 10 * phase;
      for (int c = 0; c < kShapes; ++c) {
        if (gp.count[c] == 0) continue;
        gp.launch_shape_class(c, b, s, prec);
        kinds.push_back(base + c);
        fl.push_back(gp.shape_flops[c]);
        by.push_back(gp.algo_bytes(c, prec));
        mark();
      }
      if (gp.nreduce > 0) {
        gp.launch_reduce(b, s);
        kinds.push_back(base + kShapes);
        fl.push_back(0.0);
        by.push_back(0.0);
        mark();
      }
    }
  }
  BSD_HIP(hipStreamSynchronize(s));
  int n = (int)kinds.size();
  for (int i = 0; i < n && i < cap; ++i) {
    float t = 0.f;
    BSD_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
    ms[i] = t;
    flops[i] = fl[i];
    if (bytes) bytes[i] = by[i];
    kind[i] = kinds[i];
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  return n;
}

HpsiPlan::~HpsiPlan() {
  if (side) (void)hipStreamSynchronize(side);
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  for (int i = 0; i < 2; ++i) {
    if (ev_loaded[i]) (void)hipEventDestroy(ev_loaded[i]);
    if (ev_free[i]) (void)hipEventDestroy(ev_free[i]);
  }
  if (side) (void)hipStreamDestroy(side);
  if (pack_host) (void)hipHostFree(pack_host);
}

static void stream_sleep_fn(void* arg) {
  const double ms = *static_cast<double*>(arg);
  delete static_cast<double*>(arg);
  std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(ms * 1000.0)));
}

void run_hpsi_stream(HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision,
                     double delay_ms) {
  zero_fill(out, plan.lay.n_elems, s);
  const GBases b = hpsi_bases(plan, psi, out);
  if (precision != 0) {
    const SplitTask* tasks = static_cast<const SplitTask*>(plan.split_tasks.p);
    launch_split_planes(tasks, plan.n_split_psi, b, s);
  }
  // both slots free once the work queued so far on s is done
  for (int i = 0; i < 2; ++i) BSD_HIP(hipEventRecord(plan.ev_free[i], s));
  const int n = (int)plan.phase1.size();
  auto load = [&](int k) {
    const int sl = k % 2;
    BSD_HIP(hipStreamWaitEvent(plan.side, plan.ev_free[sl], 0));
    if (delay_ms > 0) BSD_HIP(hipLaunchHostFunc(plan.side, stream_sleep_fn, new double(delay_ms)));
    const StreamChunk& sc = plan.schunks[k];
    if (sc.elems > 0)
      BSD_HIP(hipMemcpyAsync(static_cast<char*>(plan.slots.p) + (size_t)sl * plan.slot_bytes,
                             static_cast<const char*>(plan.pack_host) + sc.host_off, (size_t)sc.elems * sizeof(double),
                             hipMemcpyHostToDevice, plan.side));
    BSD_HIP(hipEventRecord(plan.ev_loaded[sl], plan.side));
  };
  if (n > 0) load(0);
  for (int k = 0; k < n; ++k) {
    const int sl = k % 2;
    BSD_HIP(hipStreamWaitEvent(s, plan.ev_loaded[sl], 0));
    // the next chunk's copy goes into the other slot while this chunk computes
    if (k + 1 < n) load(k + 1);
    if (precision == 0) {
      plan.phase1[k]->launch(b, s, 0);
      plan.phase2[k]->launch(b, s, 0);
    } else {
      const StreamChunk& sc = plan.schunks[k];
      plan.phase1h[k]->launch(b, s, 0);
      plan.phase2h[k]->launch(b, s, 0);
      if (!sc.split.empty())
        launch_split_planes(static_cast<const SplitTask*>(sc.split_dev.p), (int)sc.split.size(), b, s);
      plan.phase1s[k]->launch(b, s, precision);
      plan.phase2s[k]->launch(b, s, precision);
    }
    BSD_HIP(hipEventRecord(plan.ev_free[sl], s));
  }
}

void run_hpsi_graph(HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision) {
  if (plan.stream_r) {
    // streamed products run eagerly (copies on the side stream between chunks)
    run_hpsi_stream(plan, psi, out, s, precision, plan.stream_delay_ms);
    return;
  }
  for (auto& g : plan.graphs)
    if (g.psi == psi && g.out == out && g.precision == precision) {
      BSD_HIP(hipGraphLaunch(g.exec, s));
      return;
    }
  if (plan.graphs.size() >= 16) {
    BSD_HIP(hipStreamSynchronize(s));
    (void)hipGraphExecDestroy(plan.graphs.front().exec);
    plan.graphs.erase(plan.graphs.begin());
  }
  hipStream_t cs;
  BSD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph;
  BSD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  run_hpsi(plan, psi, out, cs, precision);
  BSD_HIP(hipStreamEndCapture(cs, &graph));
  hipGraphExec_t exec;
  BSD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  BSD_HIP(hipGraphDestroy(graph));
  BSD_HIP(hipStreamDestroy(cs));
  plan.graphs.push_back({psi, out, precision, exec});
  BSD_HIP(hipGraphLaunch(exec, s));
}

const double* hpsi_diagonal(HpsiPlan& plan, hipStream_t s) {
  if (!plan.diag_ready) {
    plan.diag.reserve(std::max<int64_t>(1, plan.lay.n_elems) * sizeof(double));
    double* d = static_cast<double*>(plan.diag.p);
    zero_fill(d, plan.lay.n_elems, s);
    GBases b{{0, 0, (uint64_t)d, 0}};
    plan.diag_plan->launch(b, s);
    plan.diag_ready = true;
  }
  return static_cast<const double*>(plan.diag.p);
}

void run_hpsi(const HpsiPlan& plan, const double* psi, double* out, hipStream_t s, int precision) {
  zero_fill(out, plan.lay.n_elems, s);
  const GBases b = hpsi_bases(plan, psi, out);
  const SplitTask* tasks = static_cast<const SplitTask*>(plan.split_tasks.p);
  if (precision != 0) launch_split_planes(tasks, plan.n_split_psi, b, s);
  for (size_t k = 0; k < plan.phase1.size(); ++k) {
    if (precision == 0) {
      plan.phase1[k]->launch(b, s, 0);
      plan.phase2[k]->launch(b, s, 0);
    } else {
      plan.phase1h[k]->launch(b, s, 0);
      plan.phase2h[k]->launch(b, s, 0);
      plan.phase1s[k]->launch(b, s, precision);
      plan.phase2s[k]->launch(b, s, precision);
    }
  }
}

}  // namespace bsd
