// Split-bf16 block products on pre-split operand planes.
//
// The float64 operands of the block GEMMs are cut once into three bf16 parts
// (x ~ h + m + l) and stored as planes whose layout is exactly the per-lane
// operand of v_mfma_f32_16x16x32_bf16 (8 consecutive K values of one row per
// lane, 16 bytes per part).  Splitting once means the product kernel only
// streams bf16 chunks and runs MFMAs; the L-operator blocks are split when the
// product is prepared, psi and the phase-1 intermediates once per product.
//
// Products kept: h h + h m + m h (3 MFMAs, float32 accuracy of the dominant
// terms) or additionally h l + m m + l h (6 MFMAs).  Every K-segment is summed
// in float32 by the MFMAs and then added, times its coefficient alpha, into
// float64 accumulators.
#include "devutil.h"

#include <algorithm>
#include <type_traits>

namespace bsd {

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(double x, unsigned short& h, unsigned short& m, unsigned short& l) {
  h = bf16_rne((float)x);
  const double r1 = x - bf16_to_double(h);
  m = bf16_rne((float)r1);
  const double r2 = r1 - bf16_to_double(m);
  l = bf16_rne((float)r2);
}

// the same for a float32 value (every step exact in float32)
__device__ __forceinline__ void split3f(float x, unsigned short& h, unsigned short& m, unsigned short& l) {
  h = bf16_rne(x);
  const float r1 = x - __uint_as_float(((unsigned int)h) << 16);
  m = bf16_rne(r1);
  const float r2 = r1 - __uint_as_float(((unsigned int)m) << 16);
  l = bf16_rne(r2);
}

// one workgroup per task; each thread writes one row of one chunk in all parts
__global__ void __launch_bounds__(256)
split_planes_kernel(const SplitTask* __restrict__ tasks, GBases bases) {
  const SplitTask t = tasks[blockIdx.x];
  const double* src = resolve(t.src, bases);
  const int n = t.rows * t.chunks;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    // consecutive threads read consecutive source addresses
    int i, c;
    if (t.trans) {
      i = e % t.rows;
      c = e / t.rows;
    } else {
      c = e % t.chunks;
      i = e / t.chunks;
    }
    const int si = t.rmap ? t.rmap[i] : i;
    u32x4_t w[kPlaneParts];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      unsigned short p[kPlaneParts][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = 8 * c + 2 * h + q;
        double x = 0.0;
        if (k < t.kcols && si >= 0) {
          const int sk = t.kmap ? t.kmap[k] : k;
          if (sk >= 0) x = t.trans ? src[(int64_t)sk * t.lds + si] : src[(int64_t)si * t.lds + sk];
        }
        split3(x, p[0][q], p[1][q], p[2][q]);
      }
#pragma unroll
      for (int pl = 0; pl < kPlaneParts; ++pl) w[pl][h] = (unsigned int)p[pl][0] | ((unsigned int)p[pl][1] << 16);
    }
#pragma unroll
    for (int pl = 0; pl < kPlaneParts; ++pl)
      *reinterpret_cast<u32x4_t*>(t.dst + plane_off(i, c, pl, t.chunks)) = w[pl];
  }
}

void launch_split_planes(const SplitTask* tasks, int n, const GBases& b, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(split_planes_kernel, dim3(n), dim3(256), 0, s, tasks, b);
  BSD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- wave tiles on planes
// Every wave owns one TW x TW output tile.  In a pass over 32 values of K the
// lane (r, q) (r = lane % 16, q = lane / 16) loads chunk 4 pass + q of its A
// rows and of its B columns; the identity operand is generated in registers.
//
// Operands arrive through buffer loads: A and B of a segment are absolute
// plane addresses, every lane keeps 32-bit byte offsets of its rows, and a
// lane outside the tile or past K gets an offset beyond the buffer, which the
// hardware answers with zeros (no branches around loads).  Descriptors are
// read with scalar loads.  Two operand sets alternate (load the next pass
// into one while the MFMAs run on the other).
typedef __attribute__((address_space(4))) const GSeg* cseg_ptr;
typedef __attribute__((address_space(4))) const GTile* ctile_ptr;

// member-wise reads through the constant address space (scalar loads for
// wave-uniform indices)
__device__ __forceinline__ GSeg ld_seg(cseg_ptr p, int i) {
  GSeg g;
  g.A = p[i].A;
  g.B = p[i].B;
  g.lda = p[i].lda;
  g.ldb = p[i].ldb;
  g.K = p[i].K;
  g.flags = p[i].flags;
  g.alpha = p[i].alpha;
  return g;
}
__device__ __forceinline__ GTile ld_tile(ctile_ptr p, int i) {
  GTile t;
  t.C = p[i].C;
  t.ldc = p[i].ldc;
  t.M = p[i].M;
  t.N = p[i].N;
  t.m0 = p[i].m0;
  t.n0 = p[i].n0;
  t.seg0 = p[i].seg0;
  t.nseg = p[i].nseg;
  t.beta = p[i].beta;
  return t;
}
constexpr unsigned kBufOut = 0x80000000u;    // byte offset past every plane buffer
constexpr int kBufFlags = 0x00020000;        // raw buffer, 32-bit data

struct PSeg {
  __amdgpu_buffer_rsrc_t ra, rb;
  int lda, ldb;      // chunks per row group
  int nch;           // chunks of K left from this step (0: empty step)
  int kbase;         // first K index of the step (identity operand)
  int m0, mt;        // rows of the tile the step was loaded for (identity operand)
  bool ident, fresh, end;
  double alpha;
};

// valid = false gives an empty step (its loads return zeros, nothing flushes)
__device__ __forceinline__ PSeg decode_step(const GSeg& g, bool valid) {
  PSeg w;
  w.ra = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(g.A), (short)0, 0x7FFFFFFF, kBufFlags);
  w.rb = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(g.B), (short)0, 0x7FFFFFFF, kBufFlags);
  w.lda = (int)g.lda;
  w.ldb = (int)g.ldb;
  w.nch = valid ? (g.K + 7) >> 3 : 0;
  w.kbase = (g.flags >> kStepPassShift) * 32;
  w.ident = g.flags & kIdentA;
  w.m0 = 0;
  w.mt = 0;
  w.fresh = g.flags & kStepFresh;
  w.end = valid && (g.flags & kStepEnd);
  w.alpha = g.alpha;
  return w;
}

// byte offset of (row, chunk q) inside a plane buffer with ld chunks per row group
__device__ __forceinline__ unsigned lane_off(int row, int q, int ld) {
  return (unsigned)(plane_off(row, q, 0, ld) * 2);
}

template <int NI, int NPL>
__device__ __forceinline__ void load_step(const PSeg& sg, const bool* rowok, const int* gi, const bool* colok,
                                          const int* gj, int q, u32x4_t (&a)[NI][NPL], u32x4_t (&b)[NI][NPL]) {
  const bool cok = q < sg.nch;
  // The loads are issued on every path (an identity operand reads zeros; its
  // h part is generated by ident_rows just before the MFMAs), so the number of
  // loads in flight is the same on every path and the compiler waits for
  // exactly one pass instead of for all of them.
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const unsigned o = (rowok[i] && cok && !sg.ident) ? lane_off(gi[i], q, sg.lda) : kBufOut;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) a[i][pl] = __builtin_amdgcn_raw_buffer_load_b128(sg.ra, o + pl * 128, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const unsigned o = (colok[j] && cok) ? lane_off(gj[j], q, sg.ldb) : kBufOut;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) b[j][pl] = __builtin_amdgcn_raw_buffer_load_b128(sg.rb, o + pl * 128, 0, 0);
  }
}

// The identity operand of a step (its loads returned zeros): the h part is
// 1.0 (bf16 0x3F80) where row == k, for the rows of the tile the step was
// loaded for.
template <int NI, int NPL>
__device__ __forceinline__ void ident_rows(const PSeg& sg, int r16, int q, u32x4_t (&a)[NI][NPL]) {
  const bool cok = q < sg.nch;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    u32x4_t h = {0u, 0u, 0u, 0u};
    const int d = sg.m0 + i * 16 + r16 - sg.kbase - 8 * q;
    const bool on = i * 16 + r16 < sg.mt && cok && d >= 0 && d < 8;
#pragma unroll
    for (int w = 0; w < 4; ++w) h[w] = (on && (d >> 1) == w) ? (0x3F80u << (16 * (d & 1))) : 0u;
    a[i][0] = h;
  }
}

__device__ __forceinline__ float4_t mfma_bf16(u32x4_t a, u32x4_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

// smallest products first (the identity's m and l parts are zero); a
// segment's first pass starts from zero instead of the running sum
// Sub-tiles at or beyond (ni, nj) lie outside the block and are skipped
// (wave-uniform bounds).
template <int NI, int NPL, int NPROD>
__device__ __forceinline__ void planes_mfma(const u32x4_t (&a)[NI][NPL], const u32x4_t (&b)[NI][NPL],
                                            float4_t (&t)[NI][NI], bool fresh, int ni = NI, int nj = NI) {
  const float4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      if (NI > 1 && (i >= ni || j >= nj)) continue;
      float4_t c;
      if (NPROD == 6) {
        c = mfma_bf16(a[i][NPL - 1], b[j][0], fresh ? zero : t[i][j]);
        c = mfma_bf16(a[i][1], b[j][1], c);
        c = mfma_bf16(a[i][0], b[j][NPL - 1], c);
        c = mfma_bf16(a[i][1], b[j][0], c);
      } else {
        c = mfma_bf16(a[i][1], b[j][0], fresh ? zero : t[i][j]);
      }
      c = mfma_bf16(a[i][0], b[j][1], c);
      c = mfma_bf16(a[i][0], b[j][0], c);
      t[i][j] = c;
    }
}

// What the epilogue of a tile needs (wave-uniform).
struct PEpi {
  uint64_t C;
  int64_t ldc;
  int mt, nt;
  double beta;
};

// tile -> lane coordinates of the loader
template <int NI, int TW>
__device__ __forceinline__ void tile_lanes(const GTile& T, int r16, bool* rowok, int* gi, bool* colok, int* gj) {
  const int mt = min(TW, T.M - T.m0), nt = min(TW, T.N - T.n0);
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    rowok[i] = i * 16 + r16 < mt;
    gi[i] = T.m0 + i * 16 + r16;
    colok[i] = i * 16 + r16 < nt;
    gj[i] = T.n0 + i * 16 + r16;
  }
}

template <int TW>
__device__ __forceinline__ PEpi tile_epi(const GTile& T) {
  PEpi e;
  e.C = T.C;
  e.ldc = T.ldc;
  e.mt = min(TW, T.M - T.m0);
  e.nt = min(TW, T.N - T.n0);
  e.beta = T.beta;
  return e;
}

// OUTP 0: C is float64 (C = beta C + result), segment sums go into float64
// accumulators.  OUTP 1: the result is split and stored as planes of C^T
// (element (r, c) goes to row c, K index r; the four rows 4 (lane / 16) + v a
// lane holds are four consecutive K values of one chunk); its sums stay in
// float32, which is all three bf16 parts can hold.
//
// Waves are persistent: wave w takes tiles w, w + W, w + 2W, ... (W waves in
// the grid) and runs one flattened sequence of (tile, step) through the two
// operand sets, so the next tile's descriptors and operands are in flight
// during the current tile's last MFMAs and its epilogue.
template <int TW, int NPROD, int OUTP>
__global__ void __launch_bounds__(256)
planes_persistent_kernel(const GTile* __restrict__ tiles_g, int ntiles, const GSeg* __restrict__ segs_g,
                         GBases bases) {
  constexpr int NI = TW / 16;
  constexpr int NPL = NPROD == 6 ? 3 : 2;  // parts read per operand
  typedef typename std::conditional<OUTP == 1, float4_t, double4_t>::type acc_t;
  const cseg_ptr segs = (cseg_ptr)segs_g;
  const ctile_ptr tiles = (ctile_ptr)tiles_g;
  const int lane = threadIdx.x & 63;
  const int W = gridDim.x * 4;
  int lt = uni(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (lt >= ntiles) return;
  const int r16 = lane & 15, q = lane >> 4;

  // loader: tile lt, step ls
  GTile T = ld_tile(tiles, lt);
  int ls = 0;
  bool rowok[NI], colok[NI];
  int gi[NI], gj[NI];
  tile_lanes<NI, TW>(T, r16, rowok, gi, colok, gj);
  bool loading = true;
  // descriptor of the loader's step: a real step, or an empty one (loads read
  // zeros, no memory access) for a tile without segments or past the last tile
  auto step_desc = [&]() -> PSeg {
    if (loading && T.nseg > 0) {
      PSeg d = decode_step(ld_seg(segs, T.seg0 + ls), true);
      d.m0 = T.m0;
      d.mt = min(TW, T.M - T.m0);
      return d;
    }
    GSeg g;
    g.A = 0;
    g.B = 0;
    g.lda = g.ldb = 0;
    g.K = 0;
    g.flags = kStepFresh | kStepEnd;
    g.alpha = 0.0;
    PSeg d = decode_step(g, false);
    d.end = loading;   // an empty tile still writes its (zero) result
    return d;
  };
  // move the loader one step on; returns whether that step ends its tile
  auto advance = [&]() {
    if (++ls < T.nseg) return;
    lt += W;
    ls = 0;
    if (lt < ntiles) {
      T = ld_tile(tiles, lt);
      tile_lanes<NI, TW>(T, r16, rowok, gi, colok, gj);
    } else {
      loading = false;
    }
  };

  float4_t t[NI][NI];
  acc_t acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) t[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  auto clear_acc = [&]() {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
  };
  auto flush = [&](double alpha) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (OUTP == 1) acc[i][j][v] += (float)alpha * t[i][j][v];
          else acc[i][j][v] += alpha * (double)t[i][j][v];
        }
  };
  typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
  auto epilogue = [&](const PEpi& e) {
    if (OUTP == 1) {
      // rows come in groups of 4 inside one chunk; mt is a multiple of 8.
      // Buffer stores: a lane outside the tile stores to the out-of-range
      // offset (dropped), so every step issues the same stores (park below).
      const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<double*>(resolve(e.C, bases)), (short)0, 0x7FFFFFFF, kBufFlags);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const int r = i * 16 + 4 * q;
          const int c = j * 16 + r16;
          unsigned short h[4], m[4], l[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) split3f(acc[i][j][v], h[v], m[v], l[v]);
          // plane row c (a column of C), K index r: parts 64 elements apart
          const unsigned o = (r < e.mt && c < e.nt) ? (unsigned)((plane_off(c, r >> 3, 0, e.ldc) + (r & 7)) * 2) : kBufOut;
          __builtin_amdgcn_raw_buffer_store_b64(u32x2_t{h[0] | ((unsigned)h[1] << 16), h[2] | ((unsigned)h[3] << 16)},
                                                rc, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(u32x2_t{m[0] | ((unsigned)m[1] << 16), m[2] | ((unsigned)m[3] << 16)},
                                                rc, o + 128, 0, 0);
          // three products never read the l part
          if (NPL == 3)
            __builtin_amdgcn_raw_buffer_store_b64(u32x2_t{l[0] | ((unsigned)l[1] << 16), l[2] | ((unsigned)l[3] << 16)},
                                                  rc, o + 256, 0, 0);
        }
    } else {
      double* C = const_cast<double*>(resolve(e.C, bases));
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // bf16 16x16x32 output: accumulator register v of lane l holds row 4 (l / 16) + v
            const int r = i * 16 + 4 * q + v;
            const int c = j * 16 + r16;
            if (r < e.mt && c < e.nt) {
              double* p = C + (int64_t)r * e.ldc + c;
              double x = acc[i][j][v];
              if (e.beta != 0.0) x += e.beta * (*p);
              *p = x;
            }
          }
    }
  };

  // a step that does not end its tile issues the epilogue's stores to the
  // out-of-range offset (dropped): every step then has the same number of
  // memory operations, and the waits before the MFMAs stay exact
  auto park = [&]() {
    if (OUTP == 1) {
      const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(nullptr, (short)0, 0, kBufFlags);
      const u32x2_t z = {0u, 0u};
#pragma unroll
      for (int k = 0; k < NI * NI * NPL; ++k) __builtin_amdgcn_raw_buffer_store_b64(z, rc, kBufOut, 0, 0);
    }
  };
  clear_acc();
  u32x4_t a0[NI][NPL], b0[NI][NPL], a1[NI][NPL], b1[NI][NPL];
  // set 0: the first step
  PSeg d0 = step_desc();
  PEpi e0 = tile_epi<TW>(T);
  load_step<NI, NPL>(d0, rowok, gi, colok, gj, q, a0, b0);
  bool te0 = max(T.nseg, 1) == 1;   // this step ends its tile
  advance();
  PSeg d1;
  PEpi e1 = e0;
  bool te1 = false;
  while (true) {
    // set 1: the next step (beyond the last tile: an empty step)
    d1 = step_desc();
    e1 = tile_epi<TW>(T);
    const bool more1 = loading;
    te1 = ls + 1 >= max(T.nseg, 1);
    load_step<NI, NPL>(d1, rowok, gi, colok, gj, q, a1, b1);
    if (loading) advance();
    if (d0.ident) ident_rows<NI, NPL>(d0, r16, q, a0);
    planes_mfma<NI, NPL, NPROD>(a0, b0, t, d0.fresh);
    if (d0.end) flush(d0.alpha);
    if (te0) {
      epilogue(e0);
      clear_acc();
    } else {
      park();
    }
    if (!more1) break;
    // set 0: the step after
    d0 = step_desc();
    e0 = tile_epi<TW>(T);
    const bool more0 = loading;
    te0 = ls + 1 >= max(T.nseg, 1);
    load_step<NI, NPL>(d0, rowok, gi, colok, gj, q, a0, b0);
    if (loading) advance();
    if (d1.ident) ident_rows<NI, NPL>(d1, r16, q, a1);
    planes_mfma<NI, NPL, NPROD>(a1, b1, t, d1.fresh);
    if (d1.end) flush(d1.alpha);
    if (te1) {
      epilogue(e1);
      clear_acc();
    } else {
      park();
    }
    if (!more0) break;
  }
}

// Float64 output (C = beta C + result), one tile per wave: the tiles are long
// split-K units and the hardware dispatcher balances them.  Segment sums are
// added into float64 accumulators.
template <int TW, int NPROD>
__global__ void __launch_bounds__(256)
wave_planes_kernel(const GTile* __restrict__ tiles_g, int ntiles, const GSeg* __restrict__ segs_g, GBases bases) {
  constexpr int NI = TW / 16;
  constexpr int NPL = NPROD == 6 ? 3 : 2;  // parts read per operand
  const cseg_ptr segs = (cseg_ptr)segs_g;
  const ctile_ptr tiles = (ctile_ptr)tiles_g;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = uni(blockIdx.x * 4 + wave);
  if (ti >= ntiles) return;
  const GTile tile = ld_tile(tiles, ti);
  const int M = tile.M, N = tile.N, m0 = tile.m0, n0 = tile.n0;
  const int seg0 = tile.seg0, nseg = tile.nseg;
  const int mt = min(TW, M - m0);
  const int nt = min(TW, N - n0);
  const int r16 = lane & 15, q = lane >> 4;
  bool rowok[NI], colok[NI];
  int gi[NI], gj[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    rowok[i] = i * 16 + r16 < mt;
    gi[i] = m0 + i * 16 + r16;
    colok[i] = i * 16 + r16 < nt;
    gj[i] = n0 + i * 16 + r16;
  }
  const int ni = (mt + 15) >> 4, nj = (nt + 15) >> 4;   // sub-tiles inside the block
  float4_t t[NI][NI];
  double4_t acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      t[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
  auto flush = [&](double alpha) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] += alpha * (double)t[i][j][v];
  };

  // steps alternate between two operand sets; raw descriptors are fetched
  // two steps ahead so their scalar loads are in flight a step early
  if (nseg > 0) {
    u32x4_t a0[NI][NPL], b0[NI][NPL], a1[NI][NPL], b1[NI][NPL];
    auto dec = [&](const GSeg& g, bool valid) {
      PSeg d = decode_step(g, valid);
      d.m0 = m0;
      d.mt = mt;
      return d;
    };
    PSeg d0 = dec(ld_seg(segs, seg0), true);
    GSeg gn = ld_seg(segs, seg0 + min(1, nseg - 1));
    load_step<NI, NPL>(d0, rowok, gi, colok, gj, q, a0, b0);
    for (int s = 0;; s += 2) {
      const PSeg d1 = dec(gn, s + 1 < nseg);
      gn = ld_seg(segs, seg0 + min(s + 2, nseg - 1));
      load_step<NI, NPL>(d1, rowok, gi, colok, gj, q, a1, b1);
      if (d0.ident) ident_rows<NI, NPL>(d0, r16, q, a0);
      planes_mfma<NI, NPL, NPROD>(a0, b0, t, d0.fresh, ni, nj);
      if (d0.end) flush(d0.alpha);
      if (s + 1 >= nseg) break;
      d0 = dec(gn, s + 2 < nseg);
      gn = ld_seg(segs, seg0 + min(s + 3, nseg - 1));
      load_step<NI, NPL>(d0, rowok, gi, colok, gj, q, a0, b0);
      if (d1.ident) ident_rows<NI, NPL>(d1, r16, q, a1);
      planes_mfma<NI, NPL, NPROD>(a1, b1, t, d1.fresh, ni, nj);
      if (d1.end) flush(d1.alpha);
      if (s + 2 >= nseg) break;
    }
  }
  double* C = const_cast<double*>(resolve(tile.C, bases));
  const double beta = tile.beta;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // bf16 16x16x32 output: accumulator register v of lane l holds row 4 (l / 16) + v
        const int r = i * 16 + 4 * q + v;
        const int c = j * 16 + r16;
        if (r < mt && c < nt) {
          double* p = C + (int64_t)r * tile.ldc + c;
          double x = acc[i][j][v];
          if (beta != 0.0) x += beta * (*p);
          *p = x;
        }
      }
}

// ---------------------------------------------------------------- workgroup tiles on planes
// One 64 x 64 tile of a float64 output (C = beta C + sum) per workgroup of four
// waves.  Wave w computes the 32 x 32 quadrant (w / 2, w % 2) as in
// wave_planes_kernel, but the operands of a step (four 16-row panels of A and
// four 16-column panels of B, every bf16 part) are fetched once for the four
// waves: each wave copies two panels straight from global memory into a ring
// of LDS stages (global_load_lds, 16 bytes per lane, no registers), kStages - 1
// steps ahead of the step being multiplied.  A lane past the block, past K or
// on an identity operand copies from a zero page instead, so every wave issues
// the same number of copies per step and a fixed vmcnt bound tells when its
// copies of a step have landed.  One barrier per step: after it, every copy of
// the step is in LDS and every wave has finished reading the stage the next
// copies overwrite.
__device__ __attribute__((aligned(16))) unsigned char g_zero_page[1024];

// Two stages: the copies of the next step run during this step's MFMAs.  More
// stages hide more latency per workgroup but cost LDS, and so workgroups per CU
// (at L=76 D=4096: 4 stages 364 ms, 3 stages 272-283 ms, 2 stages 265 ms of
// BF16X3 phase 2); two 16 KB (BF16X3) or 24 KB (BF16X6) stages keep five or
// three workgroups on a CU.
template <int NPL>
struct WgRing {
  static constexpr int kStages = 2;
  static constexpr int kCopies = 2 * NPL;                // per wave and step
  static constexpr int kStage = 8 * NPL * 1024;          // 4 A + 4 B panels, every part
};

// s_waitcnt vmcnt(n) (expcnt and lgkmcnt left alone), then lgkmcnt(0) and a
// workgroup barrier; the memory clobber keeps the compiler from moving LDS
// accesses across it
template <int N>
__device__ __forceinline__ void wg_step_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// OUTP 0: C is float64 (C = beta C + sum).  OUTP 1: the sum is split and
// stored as the planes of C^T, as planes_persistent_kernel stores it (a tile
// is one segment there, so the float64 sum holds the float32 one exactly).
// lgkmcnt(0) (this wave's LDS reads are in registers), then a workgroup barrier
__device__ __forceinline__ void wg_read_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int NPROD, int OUTP>
__global__ void __launch_bounds__(256)
wg_planes_kernel(const GTile* __restrict__ tiles_g, int ntiles, const GSeg* __restrict__ segs_g, GBases bases) {
  constexpr int NPL = NPROD == 6 ? 3 : 2;
  typedef WgRing<NPL> R;
  constexpr int S = R::kStages;
  __shared__ __attribute__((aligned(16))) unsigned char ring[S * R::kStage];
  const cseg_ptr segs = (cseg_ptr)segs_g;
  const ctile_ptr tiles = (ctile_ptr)tiles_g;
  const int ti = blockIdx.x;
  if (ti >= ntiles) return;   // the whole workgroup leaves together
  const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int r16 = lane & 15, q = lane >> 4;
  const GTile tile = ld_tile(tiles, ti);
  const int M = tile.M, N = tile.N, m0 = tile.m0, n0 = tile.n0, seg0 = tile.seg0, nst = tile.nseg;

  // copy role: op 0 copies A panels (rows), op 1 B panels (columns); panels 2h, 2h + 1
  const int op = wave >> 1, h = wave & 1;
  const int lim = op == 0 ? M - m0 : N - n0;
  const int org = op == 0 ? m0 : n0;
  bool lok[2];
  int lrow[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    lok[u] = (2 * h + u) * 16 + r16 < lim;
    lrow[u] = org + (2 * h + u) * 16 + r16;
  }
  const unsigned char* zero = g_zero_page + lane * 16;
  auto issue = [&](const GSeg& g, int stage) {
    unsigned char* dst = ring + stage * R::kStage + (op * 4 + 2 * h) * NPL * 1024;
    const int nch = (g.K + 7) >> 3;
    const bool skip = op == 0 && (g.flags & kIdentA);
    const unsigned char* base = reinterpret_cast<const unsigned char*>(op == 0 ? g.A : g.B);
    const int64_t ld = op == 0 ? g.lda : g.ldb;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool ok = lok[u] && q < nch && !skip;
      const unsigned char* src = ok ? base + plane_off(lrow[u], q, 0, ld) * 2 : zero;
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + (ok ? pl * 128 : 0)),
                                         (__attribute__((address_space(3))) void*)(dst + (u * NPL + pl) * 1024),
                                         16, 0, 0);
    }
  };

  // multiply role: quadrant (qm, qn) of the tile
  const int qm = wave >> 1, qn = wave & 1;
  const int mt = min(32, M - m0 - 32 * qm), nt = min(32, N - n0 - 32 * qn);
  const bool active = mt > 0 && nt > 0;
  const int ni = active ? (mt + 15) >> 4 : 0, nj = active ? (nt + 15) >> 4 : 0;
  float4_t t[2][2];
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      t[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    }

  // The loop runs in blocks of S steps, unrolled, so the stage of every step
  // and the ring of descriptors of the steps in flight (K, flags, alpha:
  // copied when the step's copies are issued) are fixed at compile time; one
  // descriptor is read per step, a step ahead of its use.  A tile without
  // steps reads no descriptor and writes beta C.
  if constexpr (OUTP == 0) {
    // long K (phase 2): one barrier per step, S - 1 steps in flight; the MFMAs
    // read their operands straight from the stage
    if (nst > 0) {
      int dK[S], dF[S];
      double dA[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        dK[k] = 0;
        dF[k] = 0;
        dA[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < S - 1; ++k)
        if (k < nst) {
          const GSeg g = ld_seg(segs, seg0 + k);
          issue(g, k);
          dK[k] = g.K;
          dF[k] = g.flags;
          dA[k] = g.alpha;
        }
      GSeg gl = ld_seg(segs, seg0 + min(S - 1, nst - 1));   // copies of the first iteration
      for (int s0 = 0; s0 < nst; s0 += S) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int s = s0 + j;
          if (s >= nst) break;
          // this wave's copies of step s have landed (later steps may still be in flight)
          const int ahead = min(nst - 1 - s, S - 2);
          if (ahead >= 2) wg_step_barrier<2 * R::kCopies>();
          else if (ahead == 1) wg_step_barrier<R::kCopies>();
          else wg_step_barrier<0>();
          const int jn = (j + S - 1) % S;   // stage of step s + S - 1
          const bool more = s + S - 1 < nst;
          if (more) {
            issue(gl, jn);
            dK[jn] = gl.K;
            dF[jn] = gl.flags;
            dA[jn] = gl.alpha;
          }
          if (active) {
            const unsigned char* st = ring + j * R::kStage + lane * 16;
            u32x4_t a[2][NPL], b[2][NPL];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int pl = 0; pl < NPL; ++pl) {
                a[i][pl] = *reinterpret_cast<const u32x4_t*>(st + ((2 * qm + i) * NPL + pl) * 1024);
                b[i][pl] = *reinterpret_cast<const u32x4_t*>(st + ((4 + 2 * qn + i) * NPL + pl) * 1024);
              }
            const int fl = dF[j];
            if (fl & kIdentA) {
              PSeg d;
              d.nch = (dK[j] + 7) >> 3;
              d.kbase = (fl >> kStepPassShift) * 32;
              d.m0 = m0 + 32 * qm;
              d.mt = mt;
              ident_rows<2, NPL>(d, r16, q, a);
            }
            planes_mfma<2, NPL, NPROD>(a, b, t, fl & kStepFresh, ni, nj);
            if (fl & kStepEnd) {
              const double al = dA[j];
#pragma unroll
              for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                  for (int v = 0; v < 4; ++v) acc[i][jj][v] += al * (double)t[i][jj][v];
            }
          }
          // the next step's copy descriptor: read after this step's LDS reads and
          // MFMAs are issued, so the scalar load overlaps them instead of holding
          // up the LDS reads (both count in lgkmcnt)
          if (more) gl = ld_seg(segs, seg0 + min(s + S, nst - 1));
        }
      }
    }
  } else {
    // short K (phase 1, one segment per tile): a step reads its operands from
    // its stage into registers, and once every wave has read them (second
    // barrier) the copies of step s + S go into that stage while the MFMAs
    // run, so S steps are in flight with S stages (138 vs 148 ms of BF16X3
    // phase 1 at L=76 D=4096; the second barrier costs phase 2 more than the
    // extra step in flight gains it)
    if (nst > 0) {
      int dK[S], dF[S];
      double dA[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        dK[k] = 0;
        dF[k] = 0;
        dA[k] = 0.0;
        if (k < nst) {
          const GSeg g = ld_seg(segs, seg0 + k);
          issue(g, k);
          dK[k] = g.K;
          dF[k] = g.flags;
          dA[k] = g.alpha;
        }
      }
      GSeg gl = ld_seg(segs, seg0 + min(S, nst - 1));   // copies of the first iteration
      for (int s0 = 0; s0 < nst; s0 += S) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int s = s0 + j;
          if (s >= nst) break;
          // this wave's copies of step s have landed (later steps may still be in flight)
          const int ahead = min(nst - 1 - s, S - 1);
          if (ahead >= 2) wg_step_barrier<2 * R::kCopies>();
          else if (ahead == 1) wg_step_barrier<R::kCopies>();
          else wg_step_barrier<0>();
          u32x4_t a[2][NPL], b[2][NPL];
          if (active) {
            const unsigned char* st = ring + j * R::kStage + lane * 16;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int pl = 0; pl < NPL; ++pl) {
                a[i][pl] = *reinterpret_cast<const u32x4_t*>(st + ((2 * qm + i) * NPL + pl) * 1024);
                b[i][pl] = *reinterpret_cast<const u32x4_t*>(st + ((4 + 2 * qn + i) * NPL + pl) * 1024);
              }
          }
          // every wave has its operands of step s in registers: the stage is free
          wg_read_barrier();
          const int fl = dF[j], kk = dK[j];
          const double al = dA[j];
          const bool more = s + S < nst;
          if (more) {
            issue(gl, j);
            dK[j] = gl.K;
            dF[j] = gl.flags;
            dA[j] = gl.alpha;
          }
          if (active) {
            if (fl & kIdentA) {
              PSeg d;
              d.nch = (kk + 7) >> 3;
              d.kbase = (fl >> kStepPassShift) * 32;
              d.m0 = m0 + 32 * qm;
              d.mt = mt;
              ident_rows<2, NPL>(d, r16, q, a);
            }
            planes_mfma<2, NPL, NPROD>(a, b, t, fl & kStepFresh, ni, nj);
            if (fl & kStepEnd) {
#pragma unroll
              for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                  for (int v = 0; v < 4; ++v) acc[i][jj][v] += al * (double)t[i][jj][v];
            }
          }
          if (more) gl = ld_seg(segs, seg0 + min(s + S + 1, nst - 1));
        }
      }
    }
  }
  if (!active) return;
  if (OUTP == 1) {
    // planes of C^T: quadrant rows are K indices (chunks 4 qm ..), its columns
    // plane rows (32 qn ..); the four values a lane holds are four consecutive
    // K values of one chunk (mt is a multiple of 8)
    typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(resolve(tile.C, bases)), (short)0, 0x7FFFFFFF, kBufFlags);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = i * 16 + 4 * q;
        const int c = j * 16 + r16;
        unsigned short hh[4], mm[4], ll[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) split3f((float)acc[i][j][v], hh[v], mm[v], ll[v]);
        if (r < mt && c < nt) {
          const unsigned o =
              (unsigned)((plane_off(32 * qn + c, (32 * qm + r) >> 3, 0, tile.ldc) + (r & 7)) * 2);
          __builtin_amdgcn_raw_buffer_store_b64(
              u32x2_t{hh[0] | ((unsigned)hh[1] << 16), hh[2] | ((unsigned)hh[3] << 16)}, rc, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(
              u32x2_t{mm[0] | ((unsigned)mm[1] << 16), mm[2] | ((unsigned)mm[3] << 16)}, rc, o + 128, 0, 0);
          if (NPL == 3)   // three products never read the l part
            __builtin_amdgcn_raw_buffer_store_b64(
                u32x2_t{ll[0] | ((unsigned)ll[1] << 16), ll[2] | ((unsigned)ll[3] << 16)}, rc, o + 256, 0, 0);
        }
      }
    return;
  }
  double* C = const_cast<double*>(resolve(tile.C, bases)) + (int64_t)(32 * qm) * tile.ldc + 32 * qn;
  const double beta = tile.beta;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i * 16 + 4 * q + v;
        const int c = j * 16 + r16;
        if (r < mt && c < nt) {
          double* p = C + (int64_t)r * tile.ldc + c;
          double x = acc[i][j][v];
          if (beta != 0.0) x += beta * (*p);
          *p = x;
        }
      }
}

template <int TW, int OUTP>
static void launch_planes_tw(const GTile* tiles, int ntiles, const GSeg* segs, const GBases& b, hipStream_t s,
                             int precision) {
  if (OUTP == 1) {
    // planes-out tiles are short (one segment): persistent waves, at most 2048
    // workgroups (8 per CU), each looping over its tiles
    const dim3 grid(std::min((ntiles + 3) / 4, 2048)), block(256);
    if (precision == 1)
      hipLaunchKernelGGL((planes_persistent_kernel<TW, 3, 1>), grid, block, 0, s, tiles, ntiles, segs, b);
    else
      hipLaunchKernelGGL((planes_persistent_kernel<TW, 6, 1>), grid, block, 0, s, tiles, ntiles, segs, b);
  } else {
    const dim3 grid((ntiles + 3) / 4), block(256);
    if (precision == 1)
      hipLaunchKernelGGL((wave_planes_kernel<TW, 3>), grid, block, 0, s, tiles, ntiles, segs, b);
    else
      hipLaunchKernelGGL((wave_planes_kernel<TW, 6>), grid, block, 0, s, tiles, ntiles, segs, b);
  }
}

void launch_planes_gemm(const GTile* tiles, int ntiles, int shape, const GSeg* segs, const GBases& b,
                        hipStream_t s, int precision, bool planes_out) {
  if (ntiles <= 0) return;
  BSD_CHECK(shape == 0 || shape == 4 || shape == 5, 1, "plane operands use wave or 64 x 64 workgroup tiles");
  BSD_CHECK(precision == 1 || precision == 2, 1, "plane operands are for split precision only");
  if (shape == 0) {
    if (planes_out) {
      if (precision == 1)
        hipLaunchKernelGGL((wg_planes_kernel<3, 1>), dim3(ntiles), dim3(256), 0, s, tiles, ntiles, segs, b);
      else
        hipLaunchKernelGGL((wg_planes_kernel<6, 1>), dim3(ntiles), dim3(256), 0, s, tiles, ntiles, segs, b);
    } else {
      if (precision == 1)
        hipLaunchKernelGGL((wg_planes_kernel<3, 0>), dim3(ntiles), dim3(256), 0, s, tiles, ntiles, segs, b);
      else
        hipLaunchKernelGGL((wg_planes_kernel<6, 0>), dim3(ntiles), dim3(256), 0, s, tiles, ntiles, segs, b);
    }
  } else if (shape == 4) {
    if (planes_out) launch_planes_tw<16, 1>(tiles, ntiles, segs, b, s, precision);
    else launch_planes_tw<16, 0>(tiles, ntiles, segs, b, s, precision);
  } else {
    if (planes_out) launch_planes_tw<32, 1>(tiles, ntiles, segs, b, s, precision);
    else launch_planes_tw<32, 0>(tiles, ntiles, segs, b, s, precision);
  }
  BSD_HIP(hipGetLastError());
}

}  // namespace bsd
