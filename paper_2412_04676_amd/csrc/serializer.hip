// Parallel serializer for layered block-sparse operator families (Sec. III.B.2).
//
// The stream size is exact before anything is written (the host computes it
// from the skeletons alone); on the device an exclusive wavefront prefix sum
// over block sizes gives every block its interval in the stream, so all
// workgroups then copy in complete independence into disjoint intervals of
// one contiguous buffer.  Byte format (little-endian):
//   header 64 B | family table 64 B/family | block tables 32 B/block |
//   zero pad to 256 | per family: n_layers x sum(rows*cols) float64, layer-major,
//   blocks compact row-major, zero pad to 256.
// Header: magic "BSDMRG01", u32 version=1, u32 n_families, u64 total, u64 payload,
// u64 meta, 24 zero bytes.  Family entry: u64 tag, i32 dq[2], u32 n_layers,
// u32 n_blocks, u32 esize=8, u32 0, u64 blocks_off, u64 payload_off,
// u64 layer_elems, u64 0.  Block entry: i32 q_in[2], i32 rows, i32 cols,
// u64 elem_off, u64 0.
#include "internal.h"

#include <algorithm>
#include <mutex>

namespace bsd {

namespace {

struct FamDesc {
  uint64_t tag;
  int32_t dqa, dqb;
  int32_t n_layers, n_blocks;
  int32_t blk0, pad;
  double* base;
  int64_t layer_stride;
};
struct BlkDesc {
  int32_t qa, qb, rows, cols, ld, pad;
  int64_t src_off;
};
// per-workgroup copy task: one row slice of one block, or a run of whole blocks
struct CopyTask {
  int32_t fam, layer, blk0, blk1, row0, nrows;
};

constexpr int kCopyElems = 8192;

__host__ __device__ inline int64_t align256(int64_t n) { return (n + 255) / 256 * 256; }

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// one workgroup (256 threads) per family: elem_off[b] = exclusive prefix sum of rows*cols
__global__ void __launch_bounds__(256)
scan_blocks_kernel(const FamDesc* __restrict__ fams, const BlkDesc* __restrict__ blks,
                   int64_t* __restrict__ elem_off, int64_t* __restrict__ layer_elems) {
  __shared__ int64_t wsum[4];
  __shared__ int64_t carry;
  const FamDesc f = fams[blockIdx.x];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int base = 0; base < f.n_blocks; base += 256) {
    const int b = base + threadIdx.x;
    int64_t v = 0;
    if (b < f.n_blocks) v = (int64_t)blks[f.blk0 + b].rows * blks[f.blk0 + b].cols;
    int64_t incl = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t prefix = carry;
    for (int w = 0; w < wave; ++w) prefix += wsum[w];
    if (b < f.n_blocks) elem_off[f.blk0 + b] = prefix + incl - v;
    __syncthreads();
    if (threadIdx.x == 255) carry = prefix + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) layer_elems[blockIdx.x] = carry;
}

// one wavefront: family-level exclusive prefix sum of aligned payload sizes
__global__ void __launch_bounds__(64)
family_offsets_kernel(const FamDesc* __restrict__ fams, int nf, int nb_total,
                      const int64_t* __restrict__ layer_elems, int64_t* __restrict__ payload_off) {
  const int64_t meta = align256(64 + 64 * (int64_t)nf + 32 * (int64_t)nb_total);
  int64_t carry = meta;
  for (int base = 0; base < nf; base += 64) {
    const int f = base + (int)threadIdx.x;
    const int64_t v = f < nf ? align256(fams[f].n_layers * layer_elems[f] * 8) : 0;
    const int64_t incl = wave_incl_scan(v);
    if (f < nf) payload_off[f] = carry + incl - v;
    carry += __shfl(incl, 63, 64);
  }
}

// one workgroup: header, family table, block tables, zero padding
__global__ void __launch_bounds__(256)
write_meta_kernel(const FamDesc* __restrict__ fams, const BlkDesc* __restrict__ blks, int nf,
                  int nb_total, const int64_t* __restrict__ elem_off,
                  const int64_t* __restrict__ layer_elems, const int64_t* __restrict__ payload_off,
                  unsigned char* __restrict__ out, uint64_t magic) {
  const int64_t meta = align256(64 + 64 * (int64_t)nf + 32 * (int64_t)nb_total);
  __shared__ int64_t total;
  if (threadIdx.x == 0) {
    int64_t p = nf > 0 ? payload_off[nf - 1] + align256(fams[nf - 1].n_layers * layer_elems[nf - 1] * 8) : meta;
    total = p;
    uint64_t* h = reinterpret_cast<uint64_t*>(out);
    h[0] = magic;
    reinterpret_cast<uint32_t*>(out)[2] = 1u;
    reinterpret_cast<uint32_t*>(out)[3] = (uint32_t)nf;
    h[2] = (uint64_t)p;
    h[3] = (uint64_t)(p - meta);
    h[4] = (uint64_t)meta;
    h[5] = h[6] = h[7] = 0;
  }
  __syncthreads();
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const FamDesc fd = fams[f];
    unsigned char* e = out + 64 + 64 * (int64_t)f;
    reinterpret_cast<uint64_t*>(e)[0] = fd.tag;
    reinterpret_cast<int32_t*>(e)[2] = fd.dqa;
    reinterpret_cast<int32_t*>(e)[3] = fd.dqb;
    reinterpret_cast<uint32_t*>(e)[4] = (uint32_t)fd.n_layers;
    reinterpret_cast<uint32_t*>(e)[5] = (uint32_t)fd.n_blocks;
    reinterpret_cast<uint32_t*>(e)[6] = 8u;
    reinterpret_cast<uint32_t*>(e)[7] = 0u;
    reinterpret_cast<uint64_t*>(e)[4] = (uint64_t)(64 + 64 * (int64_t)nf + 32 * (int64_t)fd.blk0);
    reinterpret_cast<uint64_t*>(e)[5] = (uint64_t)payload_off[f];
    reinterpret_cast<uint64_t*>(e)[6] = (uint64_t)layer_elems[f];
    reinterpret_cast<uint64_t*>(e)[7] = 0;
  }
  for (int b = threadIdx.x; b < nb_total; b += blockDim.x) {
    const BlkDesc bd = blks[b];
    unsigned char* e = out + 64 + 64 * (int64_t)nf + 32 * (int64_t)b;
    reinterpret_cast<int32_t*>(e)[0] = bd.qa;
    reinterpret_cast<int32_t*>(e)[1] = bd.qb;
    reinterpret_cast<int32_t*>(e)[2] = bd.rows;
    reinterpret_cast<int32_t*>(e)[3] = bd.cols;
    reinterpret_cast<uint64_t*>(e)[2] = (uint64_t)elem_off[b];
    reinterpret_cast<uint64_t*>(e)[3] = 0;
  }
  for (int64_t i = 64 + 64 * (int64_t)nf + 32 * (int64_t)nb_total + threadIdx.x; i < meta; i += blockDim.x) out[i] = 0;
  for (int f = 0; f < nf; ++f) {
    const int64_t end = payload_off[f] + fams[f].n_layers * layer_elems[f] * 8;
    const int64_t stop = (f + 1 < nf) ? payload_off[f + 1] : total;
    for (int64_t i = end + threadIdx.x; i < stop; i += blockDim.x) out[i] = 0;
  }
}

// Workgroups take copy tasks in a grid-stride loop: the bytes written do not
// depend on the grid size (a test checks 1, 7 and 1024 workgroups).
template <bool PACK>
__global__ void __launch_bounds__(256)
copy_kernel(const CopyTask* __restrict__ tasks, int ntasks, const FamDesc* __restrict__ fams,
            const BlkDesc* __restrict__ blks, const int64_t* __restrict__ elem_off,
            const int64_t* __restrict__ layer_elems, const int64_t* __restrict__ payload_off,
            unsigned char* __restrict__ stream, const int* __restrict__ status, int zero_pads) {
  if (!PACK && *status != 0) return;
  for (int ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
  const CopyTask t = tasks[ti];
  const FamDesc f = fams[t.fam];
  double* sbase = reinterpret_cast<double*>(stream + payload_off[t.fam]) + (int64_t)t.layer * layer_elems[t.fam];
  double* lbase = f.base + (int64_t)t.layer * f.layer_stride;
  for (int b = t.blk0; b < t.blk1; ++b) {
    const BlkDesc bd = blks[f.blk0 + b];
    const int r0 = (t.blk1 == t.blk0 + 1) ? t.row0 : 0;
    const int nr = (t.blk1 == t.blk0 + 1) ? t.nrows : bd.rows;
    double* s = sbase + elem_off[f.blk0 + b] + (int64_t)r0 * bd.cols;
    double* d = lbase + bd.src_off + (int64_t)r0 * bd.ld;
    const int64_t n = (int64_t)nr * bd.cols;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
      const int64_t r = e / bd.cols, c = e - r * bd.cols;
      if (PACK) s[e] = d[r * bd.ld + c];
      else d[r * bd.ld + c] = s[e];
    }
    if (!PACK && zero_pads && bd.ld > bd.cols) {
      // row padding is not in the stream: for the library's own blocks the
      // unpack writes it as zeros, so a block restored into fresh memory
      // equals the packed one entirely (caller-described families keep theirs)
      const int pad = bd.ld - bd.cols;
      const int64_t np = (int64_t)nr * pad;
      for (int64_t e = threadIdx.x; e < np; e += blockDim.x) {
        const int64_t r = e / pad, c = bd.cols + (e - r * pad);
        d[r * bd.ld + c] = 0.0;
      }
    }
  }
  }
}

// workgroups of the copy launches (0: one per copy task)
static int g_copy_grid = 0;
static unsigned copy_grid(int ntasks) {
  return (unsigned)(g_copy_grid > 0 ? std::min(g_copy_grid, ntasks) : ntasks);
}

// checks the stream's header and tables against the expected skeletons
__global__ void __launch_bounds__(256)
validate_kernel(const FamDesc* __restrict__ fams, const BlkDesc* __restrict__ blks, int nf,
                int nb_total, const int64_t* __restrict__ elem_off,
                const int64_t* __restrict__ layer_elems, const int64_t* __restrict__ payload_off,
                const unsigned char* __restrict__ in, int64_t bytes, uint64_t magic,
                int* __restrict__ status) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int64_t meta = align256(64 + 64 * (int64_t)nf + 32 * (int64_t)nb_total);
  int mybad = 0;
  if (threadIdx.x == 0) {
    const uint64_t* h = reinterpret_cast<const uint64_t*>(in);
    const uint32_t* h32 = reinterpret_cast<const uint32_t*>(in);
    int64_t total = payload_off[nf - 1 >= 0 ? nf - 1 : 0];
    total = nf > 0 ? total + align256(fams[nf - 1].n_layers * layer_elems[nf - 1] * 8) : meta;
    if (h[0] != magic || h32[2] != 1u || h32[3] != (uint32_t)nf || (int64_t)h[2] != bytes ||
        (int64_t)h[2] != total || (int64_t)h[4] != meta || (int64_t)h[3] != total - meta)
      mybad = 1;
  }
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const FamDesc fd = fams[f];
    const unsigned char* e = in + 64 + 64 * (int64_t)f;
    if (reinterpret_cast<const int32_t*>(e)[2] != fd.dqa || reinterpret_cast<const int32_t*>(e)[3] != fd.dqb ||
        reinterpret_cast<const uint32_t*>(e)[4] != (uint32_t)fd.n_layers ||
        reinterpret_cast<const uint32_t*>(e)[5] != (uint32_t)fd.n_blocks ||
        reinterpret_cast<const uint32_t*>(e)[6] != 8u ||
        reinterpret_cast<const uint64_t*>(e)[4] != (uint64_t)(64 + 64 * (int64_t)nf + 32 * (int64_t)fd.blk0) ||
        reinterpret_cast<const uint64_t*>(e)[5] != (uint64_t)payload_off[f] ||
        reinterpret_cast<const uint64_t*>(e)[6] != (uint64_t)layer_elems[f])
      mybad = 1;
  }
  for (int b = threadIdx.x; b < nb_total; b += blockDim.x) {
    const BlkDesc bd = blks[b];
    const unsigned char* e = in + 64 + 64 * (int64_t)nf + 32 * (int64_t)b;
    if (reinterpret_cast<const int32_t*>(e)[0] != bd.qa || reinterpret_cast<const int32_t*>(e)[1] != bd.qb ||
        reinterpret_cast<const int32_t*>(e)[2] != bd.rows || reinterpret_cast<const int32_t*>(e)[3] != bd.cols ||
        reinterpret_cast<const uint64_t*>(e)[2] != (uint64_t)elem_off[b])
      mybad = 1;
  }
  if (mybad) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) *status = bad ? 7 : 0;
}

uint64_t magic_word() {
  uint64_t m;
  std::memcpy(&m, "BSDMRG01", 8);
  return m;
}

}  // namespace

struct SerialPlan {
  DevBuf fams, blks, tasks, elem_off, layer_elems, payload_off, status;
  int nf = 0, nb = 0, ntasks = 0;
  int zero_pads = 0;   // unpack writes row padding as zeros (library-owned blocks)
  size_t bytes = 0;
  // host copies for the segmented form: per family its layer count, layer
  // elements, payload offset in the one-stream layout, skeleton fingerprint and
  // the first copy task of every layer (tasks are emitted family by family,
  // layer by layer, so a layer range is a contiguous task range)
  std::vector<int> h_layers;
  std::vector<int64_t> h_layer_elems, h_payload_off;
  std::vector<uint64_t> h_tag, h_print;
  std::vector<std::vector<int>> h_task_first;
};

// copy tasks of one family: large blocks in row slices, small blocks in runs
template <class Emit>
static void family_tasks(int f, int n_layers, int nbk, const int* rows, const int* cols, Emit&& emit) {
  for (int l = 0; l < n_layers; ++l) {
    int b = 0;
    while (b < nbk) {
      int64_t n = (int64_t)rows[b] * cols[b];
      if (n >= kCopyElems) {
        int rows_per = std::max(1, (int)(kCopyElems / std::max(1, cols[b])));
        for (int r0 = 0; r0 < rows[b]; r0 += rows_per) emit(CopyTask{f, l, b, b + 1, r0, std::min(rows_per, rows[b] - r0)});
        ++b;
      } else {
        int b1 = b;
        int64_t acc = 0;
        while (b1 < nbk && acc + (int64_t)rows[b1] * cols[b1] < kCopyElems) {
          acc += (int64_t)rows[b1] * cols[b1];
          ++b1;
        }
        if (b1 == b) b1 = b + 1;
        if (b1 == b + 1)
          emit(CopyTask{f, l, b, b1, 0, rows[b]});
        else
          emit(CopyTask{f, l, b, b1, 0, 0});
        b = b1;
      }
    }
  }
}

static void upload(const std::vector<FamilyView>& fv, SerialPlan& d, hipStream_t s) {
  std::vector<FamDesc> fd;
  std::vector<BlkDesc> bd;
  std::vector<CopyTask> tasks;
  for (size_t f = 0; f < fv.size(); ++f) {
    const auto& v = fv[f];
    FamDesc x;
    x.tag = v.tag;
    x.dqa = v.dq.a;
    x.dqb = v.dq.b;
    x.n_layers = v.n_layers;
    x.n_blocks = (int)v.bq.size();
    x.blk0 = (int)bd.size();
    x.pad = 0;
    x.base = static_cast<double*>(v.data);
    x.layer_stride = v.layer_stride;
    fd.push_back(x);
    for (size_t b = 0; b < v.bq.size(); ++b) {
      BlkDesc y;
      y.qa = v.bq[b].a;
      y.qb = v.bq[b].b;
      y.rows = v.rows[b];
      y.cols = v.cols[b];
      y.ld = v.ld[b];
      y.pad = 0;
      y.src_off = v.off[b];
      bd.push_back(y);
    }
    std::vector<int> first(v.n_layers + 1, (int)tasks.size());
    family_tasks((int)f, v.n_layers, (int)v.bq.size(), v.rows.data(), v.cols.data(), [&](const CopyTask& t) {
      tasks.push_back(t);
      first[t.layer + 1] = (int)tasks.size();
    });
    for (int l = 1; l <= v.n_layers; ++l) first[l] = std::max(first[l], first[l - 1]);
    int64_t le = 0;
    // 64-bit FNV-1a (offset basis 0xcbf29ce484222325, prime 0x100000001b3) over
    // the little-endian bytes of the skeleton: dq, layer count, every block's
    // sector and shape
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&](int64_t x) {
      for (int k = 0; k < 8; ++k) {
        h ^= (uint64_t)((x >> (8 * k)) & 0xff);
        h *= 0x100000001b3ull;
      }
    };
    mix(v.dq.a);
    mix(v.dq.b);
    mix(v.n_layers);
    for (size_t b = 0; b < v.bq.size(); ++b) {
      le += (int64_t)v.rows[b] * v.cols[b];
      mix(v.bq[b].a);
      mix(v.bq[b].b);
      mix(v.rows[b]);
      mix(v.cols[b]);
    }
    d.h_layers.push_back(v.n_layers);
    d.h_layer_elems.push_back(le);
    d.h_tag.push_back(v.tag);
    d.h_print.push_back(h);
    d.h_task_first.push_back(std::move(first));
  }
  {
    int64_t nbt = 0;
    for (auto& v : fv) nbt += (int64_t)v.bq.size();
    int64_t off = align256(64 + 64 * (int64_t)fv.size() + 32 * nbt);
    for (size_t f = 0; f < fv.size(); ++f) {
      d.h_payload_off.push_back(off);
      off += align256((int64_t)d.h_layers[f] * d.h_layer_elems[f] * 8);
    }
  }
  d.nf = (int)fd.size();
  d.nb = (int)bd.size();
  d.ntasks = (int)tasks.size();
  d.fams.reserve(std::max<size_t>(1, fd.size()) * sizeof(FamDesc));
  d.blks.reserve(std::max<size_t>(1, bd.size()) * sizeof(BlkDesc));
  d.tasks.reserve(std::max<size_t>(1, tasks.size()) * sizeof(CopyTask));
  d.elem_off.reserve(std::max<size_t>(1, bd.size()) * sizeof(int64_t));
  d.layer_elems.reserve(std::max<size_t>(1, fd.size()) * sizeof(int64_t));
  d.payload_off.reserve(std::max<size_t>(1, fd.size()) * sizeof(int64_t));
  d.status.reserve(256);
  if (!fd.empty()) BSD_HIP(hipMemcpyAsync(d.fams.p, fd.data(), fd.size() * sizeof(FamDesc), hipMemcpyHostToDevice, s));
  if (!bd.empty()) BSD_HIP(hipMemcpyAsync(d.blks.p, bd.data(), bd.size() * sizeof(BlkDesc), hipMemcpyHostToDevice, s));
  if (!tasks.empty())
    BSD_HIP(hipMemcpyAsync(d.tasks.p, tasks.data(), tasks.size() * sizeof(CopyTask), hipMemcpyHostToDevice, s));
  BSD_HIP(hipStreamSynchronize(s));
}

static void scan(SerialPlan& d, hipStream_t s) {
  if (d.nf > 0) {
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(d.nf), dim3(256), 0, s, (const FamDesc*)d.fams.p,
                       (const BlkDesc*)d.blks.p, (int64_t*)d.elem_off.p, (int64_t*)d.layer_elems.p);
    BSD_HIP(hipGetLastError());
    hipLaunchKernelGGL(family_offsets_kernel, dim3(1), dim3(64), 0, s, (const FamDesc*)d.fams.p, d.nf, d.nb,
                       (const int64_t*)d.layer_elems.p, (int64_t*)d.payload_off.p);
    BSD_HIP(hipGetLastError());
  }
}

size_t serialized_size(const std::vector<FamilyView>& fams) {
  int64_t nb = 0;
  for (auto& f : fams) nb += (int64_t)f.bq.size();
  int64_t total = align256(64 + 64 * (int64_t)fams.size() + 32 * nb);
  for (auto& f : fams) {
    int64_t le = 0;
    for (size_t b = 0; b < f.bq.size(); ++b) le += (int64_t)f.rows[b] * f.cols[b];
    total += align256((int64_t)f.n_layers * le * 8);
  }
  return (size_t)total;
}

void SerialPlanDeleter::operator()(SerialPlan* p) const { delete p; }

SerialPlanPtr serial_plan(const std::vector<FamilyView>& fams, hipStream_t s, bool zero_pads) {
  SerialPlanPtr p(new SerialPlan());
  p->zero_pads = zero_pads ? 1 : 0;
  p->bytes = serialized_size(fams);
  upload(fams, *p, s);
  return p;
}

size_t serial_bytes(const SerialPlan& p) { return p.bytes; }

void serial_pack(const SerialPlan& d, void* dst, size_t cap, hipStream_t s) {
  BSD_CHECK(cap >= d.bytes, 4, "destination buffer smaller than the serialized size");
  BSD_CHECK(((uintptr_t)dst % 256) == 0, 1, "destination must be 256-byte aligned");
  scan(const_cast<SerialPlan&>(d), s);
  hipLaunchKernelGGL(write_meta_kernel, dim3(1), dim3(256), 0, s, (const FamDesc*)d.fams.p,
                     (const BlkDesc*)d.blks.p, d.nf, d.nb, (const int64_t*)d.elem_off.p,
                     (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p,
                     (unsigned char*)dst, magic_word());
  BSD_HIP(hipGetLastError());
  if (d.ntasks > 0)
    hipLaunchKernelGGL((copy_kernel<true>), dim3(copy_grid(d.ntasks)), dim3(256), 0, s, (const CopyTask*)d.tasks.p,
                       d.ntasks, (const FamDesc*)d.fams.p, (const BlkDesc*)d.blks.p, (const int64_t*)d.elem_off.p,
                       (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p,
                       (unsigned char*)dst, (const int*)nullptr, 0);
  BSD_HIP(hipGetLastError());
}

void serial_unpack(const SerialPlan& d, const void* src, size_t bytes, hipStream_t s) {
  BSD_CHECK(bytes == d.bytes, 7, "stream size does not match the target skeletons");
  BSD_CHECK(((uintptr_t)src % 256) == 0, 1, "source must be 256-byte aligned");
  scan(const_cast<SerialPlan&>(d), s);
  hipLaunchKernelGGL(validate_kernel, dim3(1), dim3(256), 0, s, (const FamDesc*)d.fams.p,
                     (const BlkDesc*)d.blks.p, d.nf, d.nb, (const int64_t*)d.elem_off.p,
                     (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p,
                     (const unsigned char*)src, (int64_t)bytes, magic_word(), (int*)d.status.p);
  BSD_HIP(hipGetLastError());
  if (d.ntasks > 0)
    hipLaunchKernelGGL((copy_kernel<false>), dim3(copy_grid(d.ntasks)), dim3(256), 0, s, (const CopyTask*)d.tasks.p,
                       d.ntasks, (const FamDesc*)d.fams.p, (const BlkDesc*)d.blks.p, (const int64_t*)d.elem_off.p,
                       (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p,
                       (unsigned char*)const_cast<void*>(src), (const int*)d.status.p, d.zero_pads);
  BSD_HIP(hipGetLastError());
}

int serial_status(const SerialPlan& d, hipStream_t s) {
  int st = 0;
  BSD_HIP(hipMemcpyAsync(&st, d.status.p, sizeof(int), hipMemcpyDeviceToHost, s));
  BSD_HIP(hipStreamSynchronize(s));
  return st;
}

int validate_stream_host(const std::vector<FamilyView>& fams, const void* src, size_t bytes) {
  const size_t need = serialized_size(fams);
  if (bytes != need) return 7;
  const unsigned char* p = static_cast<const unsigned char*>(src);
  uint64_t m;
  std::memcpy(&m, p, 8);
  if (m != magic_word()) return 7;
  uint32_t ver, nf;
  std::memcpy(&ver, p + 8, 4);
  std::memcpy(&nf, p + 12, 4);
  uint64_t total;
  std::memcpy(&total, p + 16, 8);
  if (ver != 1 || nf != fams.size() || total != bytes) return 7;
  int64_t nb = 0;
  for (auto& f : fams) nb += (int64_t)f.bq.size();
  int64_t meta = align256(64 + 64 * (int64_t)fams.size() + 32 * nb);
  int64_t poff = meta, boff = 64 + 64 * (int64_t)fams.size();
  for (size_t f = 0; f < fams.size(); ++f) {
    const unsigned char* e = p + 64 + 64 * f;
    int32_t dq[2];
    uint32_t nl, nbk;
    uint64_t bo, po, le;
    std::memcpy(dq, e + 8, 8);
    std::memcpy(&nl, e + 16, 4);
    std::memcpy(&nbk, e + 20, 4);
    std::memcpy(&bo, e + 32, 8);
    std::memcpy(&po, e + 40, 8);
    std::memcpy(&le, e + 48, 8);
    int64_t lex = 0;
    for (size_t b = 0; b < fams[f].bq.size(); ++b) {
      const unsigned char* be = p + boff + 32 * b;
      int32_t bb[4];
      uint64_t eo;
      std::memcpy(bb, be, 16);
      std::memcpy(&eo, be + 16, 8);
      if (bb[0] != fams[f].bq[b].a || bb[1] != fams[f].bq[b].b || bb[2] != fams[f].rows[b] ||
          bb[3] != fams[f].cols[b] || (int64_t)eo != lex)
        return 7;
      lex += (int64_t)fams[f].rows[b] * fams[f].cols[b];
    }
    if (dq[0] != fams[f].dq.a || dq[1] != fams[f].dq.b || (int)nl != fams[f].n_layers ||
        nbk != fams[f].bq.size() || (int64_t)bo != boff || (int64_t)po != poff || (int64_t)le != lex)
      return 7;
    boff += 32 * (int64_t)nbk;
    poff += align256((int64_t)nl * lex * 8);
  }
  return poff == (int64_t)bytes ? 0 : 7;
}

// ---------------------------------------------------------------- segments
// The synchronous small-buffer form of Sec. III.A (strategy 1, Fig. 4b) with
// self-contained packages (Sec. III.B.3): a block's families are cut into
// segments of whole layers that fit half of a small device staging area; each
// segment is packed into one half while the other half is copied to pinned
// host memory, and carries a header that says where its layers belong, so a
// reader can take the segments in any order.  Segment layout (little-endian):
//   header 256 B: magic "BSDSEG01", u64 owner (the block's family tags without
//   the family index), u32 family, u32 families in the block, u32 first layer,
//   u32 layers, u64 payload bytes, u64 skeleton fingerprint of the family,
//   u64 segment index, zero to 256 B;
//   payload: the layers, blocks compact row-major, zero padded to 256 B.
namespace {
struct SegHeader {
  uint64_t magic, owner;
  uint32_t fam, nfam, layer0, nlayers;
  uint64_t payload, print, index;
};
constexpr int64_t kSegHeader = 256;
uint64_t seg_magic() {
  uint64_t m;
  std::memcpy(&m, "BSDSEG01", 8);
  return m;
}
uint64_t owner_of(const SerialPlan& d) { return d.nf ? (d.h_tag[0] & ~((1ull << 20) - 1)) : 0; }

struct SegPiece {
  int fam, l0, nl;
  int64_t bytes;
};
std::vector<SegPiece> seg_pieces(const SerialPlan& d, size_t half) {
  std::vector<SegPiece> out;
  for (int f = 0; f < d.nf; ++f) {
    const int64_t lb = d.h_layer_elems[f] * 8;
    if (lb == 0 || d.h_layers[f] == 0) continue;
    BSD_CHECK(lb <= (int64_t)half, 4, "half the staging area is smaller than one layer of a family");
    const int per = (int)std::max<int64_t>(1, (int64_t)half / lb);
    for (int l0 = 0; l0 < d.h_layers[f]; l0 += per) {
      const int nl = std::min(per, d.h_layers[f] - l0);
      out.push_back({f, l0, nl, (int64_t)nl * lb});
    }
  }
  return out;
}
}  // namespace

size_t serial_segments_size(const SerialPlan& d, size_t staging_bytes, int* nseg) {
  const size_t half = staging_bytes / 2 / 256 * 256;
  auto pcs = seg_pieces(d, half);
  size_t total = 0;
  for (auto& p : pcs) total += kSegHeader + align256(p.bytes);
  if (nseg) *nseg = (int)pcs.size();
  return total;
}

static void launch_copy_range(const SerialPlan& d, bool pack, int fam, int l0, int nl, unsigned char* buf,
                              const int* zero_status, hipStream_t s) {
  const int t0 = d.h_task_first[fam][l0], t1 = d.h_task_first[fam][l0 + nl];
  if (t1 <= t0) return;
  // the kernel adds the family's payload offset and layer offset of the
  // one-stream layout; this base makes that land in the segment buffer
  unsigned char* base = buf - (d.h_payload_off[fam] + (int64_t)l0 * d.h_layer_elems[fam] * 8);
  const CopyTask* tasks = (const CopyTask*)d.tasks.p + t0;
  if (pack)
    hipLaunchKernelGGL((copy_kernel<true>), dim3(copy_grid(t1 - t0)), dim3(256), 0, s, tasks, t1 - t0,
                       (const FamDesc*)d.fams.p, (const BlkDesc*)d.blks.p, (const int64_t*)d.elem_off.p,
                       (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p, base, (const int*)nullptr, 0);
  else
    hipLaunchKernelGGL((copy_kernel<false>), dim3(copy_grid(t1 - t0)), dim3(256), 0, s, tasks, t1 - t0,
                       (const FamDesc*)d.fams.p, (const BlkDesc*)d.blks.p, (const int64_t*)d.elem_off.p,
                       (const int64_t*)d.layer_elems.p, (const int64_t*)d.payload_off.p, base, zero_status,
                       d.zero_pads);
  BSD_HIP(hipGetLastError());
}

size_t serial_pack_segments(const SerialPlan& d, void* staging, size_t staging_bytes, void* host, size_t cap,
                            int* nseg, hipStream_t compute, hipStream_t side) {
  BSD_CHECK(((uintptr_t)staging % 256) == 0, 1, "staging must be 256-byte aligned");
  const size_t half = staging_bytes / 2 / 256 * 256;
  BSD_CHECK(half >= 256, 4, "staging area below 512 bytes");
  auto pcs = seg_pieces(d, half);
  size_t total = 0;
  for (auto& p : pcs) total += kSegHeader + align256(p.bytes);
  BSD_CHECK(cap >= total, 4, "host buffer smaller than the segmented size");
  scan(const_cast<SerialPlan&>(d), compute);
  hipEvent_t packed[2], freed[2];
  for (int i = 0; i < 2; ++i) {
    BSD_HIP(hipEventCreateWithFlags(&packed[i], hipEventDisableTiming));
    BSD_HIP(hipEventCreateWithFlags(&freed[i], hipEventDisableTiming));
    BSD_HIP(hipEventRecord(freed[i], side));
  }
  unsigned char* h = static_cast<unsigned char*>(host);
  size_t at = 0;
  for (size_t i = 0; i < pcs.size(); ++i) {
    const SegPiece& p = pcs[i];
    const int b = (int)(i % 2);
    unsigned char* buf = static_cast<unsigned char*>(staging) + (size_t)b * half;
    BSD_HIP(hipStreamWaitEvent(compute, freed[b], 0));
    launch_copy_range(d, true, p.fam, p.l0, p.nl, buf, nullptr, compute);
    BSD_HIP(hipEventRecord(packed[b], compute));
    SegHeader hd{seg_magic(), owner_of(d), (uint32_t)p.fam, (uint32_t)d.nf, (uint32_t)p.l0, (uint32_t)p.nl,
                 (uint64_t)p.bytes, d.h_print[p.fam], (uint64_t)i};
    std::memset(h + at, 0, kSegHeader);
    std::memcpy(h + at, &hd, sizeof(hd));
    const int64_t padded = align256(p.bytes);
    if (padded > p.bytes) std::memset(h + at + kSegHeader + p.bytes, 0, padded - p.bytes);
    BSD_HIP(hipStreamWaitEvent(side, packed[b], 0));
    BSD_HIP(hipMemcpyAsync(h + at + kSegHeader, buf, (size_t)p.bytes, hipMemcpyDeviceToHost, side));
    BSD_HIP(hipEventRecord(freed[b], side));
    at += kSegHeader + padded;
  }
  BSD_HIP(hipStreamSynchronize(side));
  BSD_HIP(hipStreamSynchronize(compute));
  for (int i = 0; i < 2; ++i) {
    (void)hipEventDestroy(packed[i]);
    (void)hipEventDestroy(freed[i]);
  }
  if (nseg) *nseg = (int)pcs.size();
  return total;
}

int serial_unpack_segments(const SerialPlan& d, const void* host, size_t bytes, void* staging, size_t staging_bytes,
                           hipStream_t compute, hipStream_t side) {
  BSD_CHECK(((uintptr_t)staging % 256) == 0, 1, "staging must be 256-byte aligned");
  const size_t half = staging_bytes / 2 / 256 * 256;
  // read and check every header first: nothing is written unless the
  // segments cover every layer of every family exactly once
  const unsigned char* h = static_cast<const unsigned char*>(host);
  std::vector<std::pair<size_t, SegHeader>> segs;
  std::vector<std::vector<char>> seen(d.nf);
  for (int f = 0; f < d.nf; ++f) seen[f].assign(d.h_layers[f], 0);
  size_t at = 0;
  while (at < bytes) {
    if (bytes - at < (size_t)kSegHeader) return 7;
    SegHeader hd;
    std::memcpy(&hd, h + at, sizeof(hd));
    if (hd.magic != seg_magic() || hd.owner != owner_of(d) || hd.nfam != (uint32_t)d.nf || hd.fam >= (uint32_t)d.nf)
      return 7;
    const int f = (int)hd.fam;
    if (hd.print != d.h_print[f] || hd.nlayers == 0 || (int64_t)hd.layer0 + hd.nlayers > d.h_layers[f] ||
        hd.payload != (uint64_t)((int64_t)hd.nlayers * d.h_layer_elems[f] * 8) || hd.payload > half)
      return 7;
    const size_t len = kSegHeader + align256((int64_t)hd.payload);
    if (bytes - at < len) return 7;
    for (uint32_t l = hd.layer0; l < hd.layer0 + hd.nlayers; ++l) {
      if (seen[f][l]) return 7;
      seen[f][l] = 1;
    }
    segs.push_back({at, hd});
    at += len;
  }
  for (int f = 0; f < d.nf; ++f)
    if (d.h_layer_elems[f] > 0)
      for (char c : seen[f])
        if (!c) return 7;
  scan(const_cast<SerialPlan&>(d), compute);
  BSD_HIP(hipMemsetAsync(d.status.p, 0, sizeof(int), compute));
  hipEvent_t loaded[2], freed[2];
  for (int i = 0; i < 2; ++i) {
    BSD_HIP(hipEventCreateWithFlags(&loaded[i], hipEventDisableTiming));
    BSD_HIP(hipEventCreateWithFlags(&freed[i], hipEventDisableTiming));
    BSD_HIP(hipEventRecord(freed[i], compute));
  }
  for (size_t i = 0; i < segs.size(); ++i) {
    const SegHeader& hd = segs[i].second;
    const int b = (int)(i % 2);
    unsigned char* buf = static_cast<unsigned char*>(staging) + (size_t)b * half;
    BSD_HIP(hipStreamWaitEvent(side, freed[b], 0));
    BSD_HIP(hipMemcpyAsync(buf, h + segs[i].first + kSegHeader, (size_t)hd.payload, hipMemcpyHostToDevice, side));
    BSD_HIP(hipEventRecord(loaded[b], side));
    BSD_HIP(hipStreamWaitEvent(compute, loaded[b], 0));
    launch_copy_range(d, false, (int)hd.fam, (int)hd.layer0, (int)hd.nlayers, buf, (const int*)d.status.p, compute);
    BSD_HIP(hipEventRecord(freed[b], compute));
  }
  BSD_HIP(hipStreamSynchronize(compute));
  BSD_HIP(hipStreamSynchronize(side));
  for (int i = 0; i < 2; ++i) {
    (void)hipEventDestroy(loaded[i]);
    (void)hipEventDestroy(freed[i]);
  }
  return 0;
}

void set_copy_grid(int workgroups) { g_copy_grid = std::max(0, workgroups); }

// ---------------------------------------------------------------- no-allocation pack
// A pack of caller-described families that allocates nothing: the descriptor
// tables live in a file-scope device array (one per GPU, kept until the
// process ends) and are staged through a file-scope host array.  Calls are
// serialized by a mutex and synchronize their stream before returning, so
// every call finds the array free; the kernels overwrite every table entry
// they read, so nothing has to start at zero.
namespace {
constexpr size_t kNoAllocScratch = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratch];
std::mutex g_noalloc_mu;
void* g_scratch_dev[kMaxDevices] = {};
alignas(256) unsigned char g_noalloc_host[kNoAllocScratch];

size_t al256(size_t n) { return (n + 255) / 256 * 256; }
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratch; }

// the device address of this GPU's copy of `scratch` (looked up once per device)
static void* scratch_on_current_device() {
  int dev = 0;
  BSD_HIP(hipGetDevice(&dev));
  BSD_CHECK(dev >= 0 && dev < kMaxDevices, 1, "device index out of range");
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    BSD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BSD_CHECK(p != nullptr, 5, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

void pack_desc_noalloc(int nf, const FamilyDescIn* fams, void* dst, size_t cap, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  BSD_CHECK(nf >= 0 && (nf == 0 || fams != nullptr), 1, "bad family list");
  BSD_CHECK(dst != nullptr && ((uintptr_t)dst % 256) == 0, 1, "destination must be 256-byte aligned");
  // sizes first: blocks, copy tasks and the exact stream size
  int64_t nb = 0, nt = 0, payload = 0;
  for (int f = 0; f < nf; ++f) {
    const FamilyDescIn& x = fams[f];
    BSD_CHECK(x.n_layers >= 0 && x.n_blocks >= 0, 1, "negative family sizes");
    BSD_CHECK(x.n_blocks == 0 || (x.block_q && x.rows && x.cols && x.ld && x.elem_offset), 1, "missing block arrays");
    BSD_CHECK(x.n_layers == 0 || x.n_blocks == 0 || x.data != nullptr, 1, "missing data pointer");
    BSD_CHECK(((uintptr_t)x.data % 16) == 0, 1, "family data must be 16-byte aligned");
    int64_t le = 0, maxend = 0;
    for (int b = 0; b < x.n_blocks; ++b) {
      BSD_CHECK(x.rows[b] >= 0 && x.cols[b] >= 0 && x.ld[b] >= x.cols[b] && x.elem_offset[b] >= 0, 1,
                "bad block geometry");
      le += (int64_t)x.rows[b] * x.cols[b];
      if (x.rows[b] > 0)
        maxend = std::max<int64_t>(maxend, x.elem_offset[b] + (int64_t)(x.rows[b] - 1) * x.ld[b] + x.cols[b]);
    }
    BSD_CHECK(x.n_layers <= 1 || x.layer_stride >= maxend, 1, "layers overlap");
    nb += x.n_blocks;
    payload += align256((int64_t)x.n_layers * le * 8);
    family_tasks(f, x.n_layers, x.n_blocks, x.rows, x.cols, [&](const CopyTask&) { ++nt; });
  }
  const size_t bytes = (size_t)(align256(64 + 64 * (int64_t)nf + 32 * nb) + payload);
  BSD_CHECK(cap >= bytes, 4, "destination smaller than the serialized size");
  const size_t o_b = al256((size_t)nf * sizeof(FamDesc));
  const size_t o_t = o_b + al256((size_t)nb * sizeof(BlkDesc));
  const size_t o_eo = o_t + al256((size_t)nt * sizeof(CopyTask));
  const size_t o_le = o_eo + al256((size_t)nb * sizeof(int64_t));
  const size_t o_po = o_le + al256((size_t)nf * sizeof(int64_t));
  const size_t end = o_po + al256((size_t)nf * sizeof(int64_t));
  BSD_CHECK(end <= kNoAllocScratch, 1,
            "descriptor tables (" + std::to_string(end) + " bytes) exceed the no-allocation scratch of " +
                std::to_string(kNoAllocScratch) + " bytes; use bsdmrg_pack_desc");
  unsigned char* dev = static_cast<unsigned char*>(scratch_on_current_device());
  FamDesc* fd = reinterpret_cast<FamDesc*>(g_noalloc_host);
  BlkDesc* bd = reinterpret_cast<BlkDesc*>(g_noalloc_host + o_b);
  CopyTask* td = reinterpret_cast<CopyTask*>(g_noalloc_host + o_t);
  int64_t bi = 0, ti = 0;
  for (int f = 0; f < nf; ++f) {
    const FamilyDescIn& x = fams[f];
    FamDesc y;
    y.tag = x.tag;
    y.dqa = x.dq[0];
    y.dqb = x.dq[1];
    y.n_layers = x.n_layers;
    y.n_blocks = x.n_blocks;
    y.blk0 = (int)bi;
    y.pad = 0;
    y.base = static_cast<double*>(x.data);
    y.layer_stride = x.layer_stride;
    fd[f] = y;
    for (int b = 0; b < x.n_blocks; ++b) {
      BlkDesc z;
      z.qa = x.block_q[2 * b];
      z.qb = x.block_q[2 * b + 1];
      z.rows = x.rows[b];
      z.cols = x.cols[b];
      z.ld = x.ld[b];
      z.pad = 0;
      z.src_off = x.elem_offset[b];
      bd[bi++] = z;
    }
    family_tasks(f, x.n_layers, x.n_blocks, x.rows, x.cols, [&](const CopyTask& t) { td[ti++] = t; });
  }
  if (o_eo > 0) BSD_HIP(hipMemcpyAsync(dev, g_noalloc_host, o_eo, hipMemcpyHostToDevice, s));
  const FamDesc* dfd = reinterpret_cast<const FamDesc*>(dev);
  const BlkDesc* dbd = reinterpret_cast<const BlkDesc*>(dev + o_b);
  const CopyTask* dtd = reinterpret_cast<const CopyTask*>(dev + o_t);
  int64_t* eo = reinterpret_cast<int64_t*>(dev + o_eo);
  int64_t* le = reinterpret_cast<int64_t*>(dev + o_le);
  int64_t* po = reinterpret_cast<int64_t*>(dev + o_po);
  if (nf > 0) {
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(nf), dim3(256), 0, s, dfd, dbd, eo, le);
    BSD_HIP(hipGetLastError());
    hipLaunchKernelGGL(family_offsets_kernel, dim3(1), dim3(64), 0, s, dfd, nf, (int)nb, (const int64_t*)le, po);
    BSD_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(write_meta_kernel, dim3(1), dim3(256), 0, s, dfd, dbd, nf, (int)nb, (const int64_t*)eo,
                     (const int64_t*)le, (const int64_t*)po, (unsigned char*)dst, magic_word());
  BSD_HIP(hipGetLastError());
  if (nt > 0)
    hipLaunchKernelGGL((copy_kernel<true>), dim3(copy_grid((int)nt)), dim3(256), 0, s, dtd, (int)nt, dfd, dbd,
                       (const int64_t*)eo,
                       (const int64_t*)le, (const int64_t*)po, (unsigned char*)dst, (const int*)nullptr, 0);
  BSD_HIP(hipGetLastError());
  BSD_HIP(hipStreamSynchronize(s));
}

}  // namespace bsd
