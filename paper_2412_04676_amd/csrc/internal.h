// Internal declarations of the block-sparse DMRG library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace bsd {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
void set_last_error(const std::string& m);

#define BSD_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::bsd::Error(5, std::string("HIP error ") + hipGetErrorString(e_) +     \
                                " at " __FILE__ ":" + std::to_string(__LINE__));    \
  } while (0)

#define BSD_CHECK(cond, code, msg)          \
  do {                                      \
    if (!(cond)) throw ::bsd::Error(code, msg); \
  } while (0)

// ---------------------------------------------------------------- quantum numbers
struct Q {
  int a = 0, b = 0;
  bool operator<(const Q& o) const { return a != o.a ? a < o.a : b < o.b; }
  bool operator==(const Q& o) const { return a == o.a && b == o.b; }
  bool operator!=(const Q& o) const { return !(*this == o); }
  Q operator+(const Q& o) const { return {a + o.a, b + o.b}; }
  Q operator-(const Q& o) const { return {a - o.a, b - o.b}; }
  Q operator-() const { return {-a, -b}; }
  int parity() const { return ((a + b) % 2 + 2) % 2; }
};
inline Q mode_q(int p) { return (p % 2 == 0) ? Q{1, 0} : Q{0, 1}; }
extern const Q kSiteQ[4];

// ---------------------------------------------------------------- integrals
struct Integrals {
  int L = 0;
  std::vector<double> h, eri;  // h[L*L], eri[L^4] chemists' order
  double t(int p, int q) const {
    return (p % 2 == q % 2) ? h[(size_t)(p / 2) * L + q / 2] : 0.0;
  }
  // g_pqrs = (i_p i_s | i_q i_r) for sigma_p = sigma_s and sigma_q = sigma_r
  double g(int p, int q, int r, int s) const {
    if (p % 2 != s % 2 || q % 2 != r % 2) return 0.0;
    size_t ip = p / 2, is = s / 2, iq = q / 2, ir = r / 2, l = L;
    return eri[((ip * l + is) * l + iq) * l + ir];
  }
};

// ---------------------------------------------------------------- small dense local matrices
struct Mat {
  int n = 0;
  std::vector<double> a;
  Mat() {}
  explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * n + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * n + j]; }
  bool zero() const {
    for (double v : a)
      if (v != 0.0) return false;
    return true;
  }
};
Mat mat_mul(const Mat& x, const Mat& y);
Mat mat_T(const Mat& x);
Mat mat_scale(const Mat& x, double c);
void mat_axpy(Mat& y, double c, const Mat& x);
Mat mat_eye(int n);

// A set of consecutive sites treated exactly (one site for renormalization,
// two sites for the two-site superblock).  State index = sum s_k 4^(n-1-k).
struct SiteSet {
  int first = 0, nsites = 0, dim = 0;
  std::vector<Mat> cd;         // creation matrix per local mode (2*nsites)
  std::vector<Q> q;            // quantum number per state
  int mode0() const { return 2 * first; }
  int nmodes() const { return 2 * nsites; }
  bool has(int p) const { return p >= mode0() && p < mode0() + nmodes(); }
  const Mat& CD(int p) const { return cd[p - mode0()]; }
  Mat C(int p) const { return mat_T(cd[p - mode0()]); }
};
SiteSet make_siteset(int first, int nsites);

// ---------------------------------------------------------------- operator keys
// kinds: 'I' identity, 'H' block Hamiltonian, 'c' creation a+_p, 'A' a+_p a+_q (p<q),
// 'B' a+_p a_q, 'S' three-operator complementary op, 'P' and 'Q' two-index
// complementary ops.
struct OpKey {
  char kind = 'I';
  int p = -1, q = -1;
  bool operator<(const OpKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (p != o.p) return p < o.p;
    return q < o.q;
  }
  bool operator==(const OpKey& o) const { return kind == o.kind && p == o.p && q == o.q; }
};

// a term coef * op(key) with op = transpose if trans
struct Term {
  double coef;
  OpKey key;
  bool trans;
};
// sum_k terms_k (x) M : block part aggregated, local part M (dim x dim)
struct Group {
  Mat M;
  std::vector<Term> terms;
};

// Operators of an enlarged block L . C in the left (normal) role, C on the right.
std::vector<Group> expand_left(const OpKey& key, int nL_modes, const SiteSet& C,
                               const Integrals& I);
// Operators of s . R in the right role, s on the left.  R holds either the
// complementary set (H, a+_r, S_x, P_pq, Q_pq) or, with R_normal, the normal
// set of its own modes (H, a+_r, a+_r a+_s, a+_r a_s) plus S_x; then every
// complementary two-index operator of R is written as its sum over R's normal
// operators.  Keys 'A' and 'B' (new normal operators) need R_normal.
std::vector<Group> expand_right(const OpKey& key, const SiteSet& s, int R_mode0, int nmodes,
                                const Integrals& I, bool R_normal = false);
// Transpose of an expanded operator (graded: sign (-1)^{|M| |O|}).
std::vector<Group> transpose_groups(const std::vector<Group>& g, const SiteSet& C,
                                    int op_parity_of_block);
// dq of a block operator key in the given role (left: normal set, right: complementary set)
Q key_dq(const OpKey& k, bool left_block);
int local_parity(const Mat& M, const SiteSet& C);  // parity of a local operator (-1 if zero)

// ---------------------------------------------------------------- block-sparse structures
struct Basis {
  std::vector<Q> q;
  std::vector<int> dim;
  std::map<Q, int> index;
  int find(const Q& x) const {
    auto it = index.find(x);
    return it == index.end() ? -1 : it->second;
  }
  void add(const Q& x, int d) {
    index[x] = (int)q.size();
    q.push_back(x);
    dim.push_back(d);
  }
  int64_t total() const {
    int64_t s = 0;
    for (int d : dim) s += d;
    return s;
  }
};

// one dense block of a skeleton: rows x cols at element offset off (row-major, ld)
struct SkBlock {
  int in, out;   // basis indices
  int rows, cols, ld;
  int64_t off;
};
struct Skeleton {
  Q dq;
  std::vector<SkBlock> blocks;
  std::vector<int> by_in;   // basis index -> block index or -1
  int64_t layer_stride = 0; // elements per layer (multiple of 32)
};
Skeleton make_skeleton(const Basis& in, const Basis& out, const Q& dq);

// layered operators sharing one skeleton (one device allocation)
struct Family {
  Skeleton sk;
  std::vector<OpKey> keys;
  double* dev = nullptr;
  size_t bytes() const { return (size_t)sk.layer_stride * keys.size() * sizeof(double); }
};

struct OpRef {
  int fam = -1, layer = -1;
};

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf();
  void reserve(size_t bytes);
  void release();
};

// Device memory of one renormalized block: one virtual address range whose
// physical backing can be released and created again at the same address
// (HIP virtual memory management), so product plans and serializer
// descriptors that hold pointers into the block stay valid across an offload
// that frees the memory and the prefetch that restores it.  Devices without
// virtual memory management get a plain allocation; its address changes when
// it is created again (stable() reports which).
struct BlockMem {
  void* va = nullptr;
  size_t bytes = 0, reserved = 0, piece = 0;
  bool vmm = false, mapped = false;
  std::vector<uint64_t> handles;   // hipMemGenericAllocationHandle_t, one per piece of the range
  int device = 0;
  bool map_pieces();               // false (nothing left mapped) if a piece cannot be created or mapped
  BlockMem() {}
  BlockMem(const BlockMem&) = delete;
  BlockMem& operator=(const BlockMem&) = delete;
  ~BlockMem();
  void create(size_t bytes);     // reserve and back with physical memory
  void release_physical();       // frees the physical memory (no work may still use it)
  void acquire_physical();       // backs the range again (contents undefined)
  bool stable() const { return vmm; }
};

struct SerialPlan;
struct SerialPlanDeleter {
  void operator()(SerialPlan* p) const;
};
using SerialPlanPtr = std::unique_ptr<SerialPlan, SerialPlanDeleter>;

// A renormalized block with its operator families on the device.
struct Block {
  bool left = true;
  bool normal = false;       // right block holding normal operators of its own modes
  int first = 0, last = 0;   // sites [first, last)
  Basis basis;               // electrons inside the block
  std::vector<Family> fams;
  std::map<OpKey, OpRef> ops;
  std::unique_ptr<BlockMem> mem;   // every family's layers, at 256-byte aligned offsets
  std::vector<size_t> fam_off;     // byte offset of each family in mem
  bool resident = true;
  // serializer descriptors and offload state
  SerialPlanPtr splan;
  hipEvent_t offload_done = nullptr;
  hipEvent_t prefetch_done = nullptr;   // recorded on the compute stream after the unpack
  hipEvent_t last_use = nullptr;        // recorded after the last asynchronous work that reads the block
  bool offload_pending = false, release_after = false, prefetch_pending = false;
  void mark_use(hipStream_t s);         // record last_use on s
  void quiesce();                       // wait for every recorded use, copy and unpack
  ~Block();
  const double* op_block(const OpKey& k, int in_idx, int* rows, int* cols, int* ld) const;
  size_t device_bytes() const;
};

// ---------------------------------------------------------------- grouped GEMM
// Pointers are tagged: bits 56..63 select a base (0 absolute, 1 psi-in, 2 out, 3 spare).
constexpr int kTagShift = 56;
inline uint64_t tag_ptr(int cls, uint64_t off) { return ((uint64_t)cls << kTagShift) | off; }
enum { kTransA = 1, kTransB = 2, kIdentA = 4 };
// Plane-operand lists are expanded into steps of one pass (32 values of K):
// a step's A and B point at its first chunk, K counts the values left from
// there, flags carry kIdentA, kStepFresh (first pass of its segment: start a
// new sum), kStepEnd (last pass: add alpha times the sum into the tile) and,
// from bit kStepPassShift on, the pass index (for the identity operand).
enum { kStepFresh = 8, kStepEnd = 16, kStepPassShift = 8 };

struct GSeg {
  uint64_t A, B;
  int64_t lda, ldb;
  int32_t K, flags;
  double alpha;
};
// One unit of work of a grouped-GEMM launch: the tile at (m0, n0) of an M x N
// problem over the K-segments seg0 .. seg0 + nseg - 1.  C points at the tile's
// own origin: inside the problem's output, or, for one part of a split-K tile,
// at a dense workspace slot (ldc = tile width, beta = 0) that a reduction adds
// into the output afterwards.
struct GTile {
  uint64_t C;
  int64_t ldc;
  int32_t M, N, m0, n0;
  int32_t seg0, nseg;
  double beta;
};
// Fixed-order sum of the split-K parts of one tile: C = beta C + sum_p part_p.
struct GReduce {
  uint64_t C;
  int64_t ldc;
  const double* parts;
  int32_t rows, cols, nparts, ldp;
  int64_t part_stride;
  double beta;
};
struct GBases {
  uint64_t b[4];
};

// a list of output matrices, each with its own list of K-segments
struct GemmProblem {
  uint64_t C;
  int64_t ldc;
  int M, N;
  double beta;
  std::vector<GSeg> segs;
  // locality group (>= 0): problems of one group share operands and are placed
  // on one XCD, in the order of their segment lists; -1: no grouping
  int group = -1;
};

// Device-resident tile/segment lists for one launch group (64x64 and 32x32 tiles).
// Tile shape classes of the grouped GEMM: 0 64x64, 1 32x32, 2 32x64, 3 64x32
// (workgroup tiles staged through LDS), 4 16x16 and 5 32x32 (one wave each,
// float64 only).
constexpr int kShapes = 6;
// Split-bf16 operand planes.  A float64 matrix X (rows x K) is stored once as
// bf16 parts X ~ h + m + l (h = bf16(X), m = bf16(X - h), l = bf16(X - h - m)),
// laid out for the MFMA operand fetch: K is cut into chunks of 8 consecutive
// values, rows into groups of 8, and one (row group, chunk, part) is a 128-byte
// line holding the 8 x 8 values row by row:
//   element (i, k, part p) at (((i / 8) * chunks + k / 8) * 3 + p) * 64 + (i % 8) * 8 + k % 8.
// An MFMA operand load (16 rows x 4 chunks, 16 bytes per lane) then reads 8
// whole lines.  Values past K (and columns that kmap sends to -1) are zero;
// rows are padded to a multiple of 8 (padding rows are never read).
constexpr int kPlaneParts = 3;
__host__ __device__ inline int64_t plane_off(int i, int c, int p, int64_t chunks) {
  return ((((int64_t)(i >> 3) * chunks + c) * kPlaneParts + p) << 6) + ((i & 7) << 3);
}
inline int64_t plane_elems(int rows, int chunks) { return (int64_t)((rows + 7) / 8) * chunks * kPlaneParts * 64; }
struct SplitTask {
  uint64_t src;         // tagged float64 source
  int64_t lds;          // source leading dimension
  const int32_t* kmap;  // optional: plane column -> source column (-1 = zero)
  const int32_t* rmap;  // optional: plane row -> source row (-1 = zero row)
  uint16_t* dst;
  int32_t rows, kcols;  // plane rows; plane columns (source K, or kmap length)
  int32_t chunks;       // chunks per plane row (>= ceil(kcols / 8))
  int32_t trans;        // source element (i, k) at src[k * lds + i] (else src[i * lds + k])
};
void launch_split_planes(const SplitTask* tasks, int n, const GBases& b, hipStream_t s);

struct GemmBuildOpts {
  bool wave_tiles = true;      // float64 lists: blocks up to wave_max x wave_max get wave tiles;
  int wave_max = 64;           // plane lists: blocks above wave_max in both dimensions get 64 x 64 workgroup tiles
  bool split_k = true;         // cut long tiles so that every launch fills the device
  double target_waves = 8192;  // split-K: about this many waves per launch ...
  double min_part_work = 640;  // ... with parts of at least this work (sum of K + 16 per segment)
  bool xcd_order = true;       // place problems of one locality group on one XCD
  bool plane_operands = false; // A and B are split-bf16 planes (wave tiles for every size)
  bool plane_output = false;   // C is written as split-bf16 planes of C^T (M a multiple of 8)
  hipStream_t upload = nullptr; // non-null: lists are copied on this stream (then synchronized)
};

struct GemmPlan {
  int first[kShapes] = {0, 0, 0, 0, 0, 0}, count[kShapes] = {0, 0, 0, 0, 0, 0};
  bool wave = false;
  // planes: the segments' A and B point at split-bf16 planes (A rows of op(A),
  // B rows of op(B)^T, lda / ldb in chunks); launched only at split precision.
  // planes_out: the result is stored as planes of C^T (row n of C^T = column n
  // of C, ldc in chunks), the operand layout of a following planes product.
  bool planes = false, planes_out = false;
  DevBuf tiles, segs;
  // float64 wave-tile classes read their segments as steps of 16 values of K
  // (pointers advanced, K counted from the step, identity offset in the flags)
  DevBuf steps;
  // split-K: parts of long tiles write workspace slots, summed by one reduction
  DevBuf parts, reduces;
  int nreduce = 0;
  double flops = 0.0;                       // useful flops (2 M N K over non-identity segments)
  double shape_flops[kShapes] = {0, 0, 0, 0, 0, 0};
  // algorithmic HBM traffic per shape class: distinct operand blocks read once
  // (float64 values, or values per bf16 part for plane operands) and the output
  double shape_in_elems[kShapes] = {0, 0, 0, 0, 0, 0}, shape_out_bytes[kShapes] = {0, 0, 0, 0, 0, 0};
  double algo_bytes(int c, int precision) const {
    const double per = planes ? 2.0 * (precision == 1 ? 2 : kPlaneParts) : 8.0;
    return shape_in_elems[c] * per + shape_out_bytes[c];
  }
  // wave_tiles: small problems get wave tiles (the list is then float64 only);
  // split_k: cut long tiles into parts so that every launch fills the device
  void build(const std::vector<GemmProblem>& probs, const GemmBuildOpts& opts);
  void build(const std::vector<GemmProblem>& probs, bool wave_tiles = true) {
    GemmBuildOpts o;
    o.wave_tiles = wave_tiles;
    build(probs, o);
  }
  // precision: 0 float64 MFMA, 1 split-bf16 (3 products), 2 split-bf16 (6 products)
  void launch(const GBases& bases, hipStream_t s, int precision = 0) const;
  void launch_shape_class(int c, const GBases& bases, hipStream_t s, int precision = 0) const;
  void launch_reduce(const GBases& bases, hipStream_t s) const;
};

struct AggTerm {
  const double* in;
  int64_t ldi;
  int32_t flags;  // kTransA: read transposed, kIdentA: identity
  int32_t pad;
  double coef;
};
struct AggTask {
  double* out;
  int64_t ldo;
  int32_t rows, cols;
  int32_t t0, nt;
  int32_t col_major;   // walk the block column by column (most terms are read transposed)
  int32_t pad;
};
void launch_aggregate(const AggTask* tasks_dev, const AggTerm* terms_dev, int ntasks,
                      hipStream_t s);
void launch_grouped_gemm(const GTile* tiles, int ntiles, int shape, const GSeg* segs,
                         const GBases& b, hipStream_t s, int precision = 0);
void launch_split_reduce(const GReduce* red, int n, const GBases& b, hipStream_t s);
// Runs fn(i, upload) for i in [0, n) on a pool of host threads (at most 16),
// each with a non-blocking stream of its own for copies; rethrows the first
// failure after all threads have finished.
void parallel_jobs(int n, const std::function<void(int, hipStream_t)>& fn);
void launch_planes_gemm(const GTile* tiles, int ntiles, int shape, const GSeg* segs, const GBases& b,
                        hipStream_t s, int precision, bool planes_out);

// ---------------------------------------------------------------- serializer
struct FamilyView {
  uint64_t tag;
  Q dq;
  int n_layers;
  std::vector<Q> bq;
  std::vector<int> rows, cols, ld;
  std::vector<int64_t> off;
  int64_t layer_stride;
  void* data;
};
size_t serialized_size(const std::vector<FamilyView>& fams);
// device descriptors of a set of families (built once; synchronizes s)
SerialPlanPtr serial_plan(const std::vector<FamilyView>& fams, hipStream_t s, bool zero_pads = false);
size_t serial_bytes(const SerialPlan& p);
void serial_pack(const SerialPlan& p, void* dst, size_t cap, hipStream_t s);          // stream-ordered
void serial_unpack(const SerialPlan& p, const void* src, size_t bytes, hipStream_t s);  // stream-ordered
int serial_status(const SerialPlan& p, hipStream_t s);  // synchronizes s; 0 or 7 (corrupt)
int validate_stream_host(const std::vector<FamilyView>& fams, const void* src, size_t bytes);
// segmented, order-free form through a small double-buffered staging area
size_t serial_segments_size(const SerialPlan& d, size_t staging_bytes, int* nseg);
size_t serial_pack_segments(const SerialPlan& d, void* staging, size_t staging_bytes, void* host, size_t cap,
                            int* nseg, hipStream_t compute, hipStream_t side);   // synchronizing
int serial_unpack_segments(const SerialPlan& d, const void* host, size_t bytes, void* staging, size_t staging_bytes,
                           hipStream_t compute, hipStream_t side);   // synchronizing; 0 or 7 (nothing written)
void set_copy_grid(int workgroups);   // 0: one workgroup per copy task
// The caller-described family of the C ABI (same layout as bsdmrg_family_desc).
struct FamilyDescIn {
  uint64_t tag;
  int32_t dq[2];
  int32_t n_layers, n_blocks;
  const int32_t* block_q;
  const int32_t* rows;
  const int32_t* cols;
  const int32_t* ld;
  const int64_t* elem_offset;
  int64_t layer_stride;
  void* data;
};
// Pack without any allocation (device tables in a file-scope array of
// noalloc_scratch_bytes()); synchronizes s.
void pack_desc_noalloc(int n, const FamilyDescIn* fams, void* dst, size_t cap, hipStream_t s);
size_t noalloc_scratch_bytes();

}  // namespace bsd
