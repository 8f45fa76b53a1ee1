// far_internal.h -- shared internals of the gfx950 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "far.h"

namespace far {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
far_status_t hip_fail(hipError_t e, const char* what, const char* file, int line);

#define FAR_HIP(call)                                                        \
  do {                                                                       \
    hipError_t far_e_ = (call);                                              \
    if (far_e_ != hipSuccess) return far::hip_fail(far_e_, #call, __FILE__, __LINE__); \
  } while (0)

#define FAR_TRY(call)                                                        \
  do {                                                                       \
    far_status_t far_s_ = (call);                                            \
    if (far_s_ != FAR_OK) return far_s_;                                     \
  } while (0)

inline hipStream_t S(far_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- timing
// Event timing of selected launches (far_timing_enable / far_timing_read_kind).
// A TimedScope records an event on the stream at construction and one at
// destruction when timing is on; far_timing_read_kind sums the intervals.
bool timing_on();
void timing_push(int kind, hipEvent_t ev0, hipEvent_t ev1);

struct TimedScope {
  int kind;
  hipStream_t st;
  hipEvent_t ev0 = nullptr;
  TimedScope(int k, hipStream_t s) : kind(k), st(s) {
    // kind < 0: not timed (no event is created)
    if (k >= 0 && timing_on() && hipEventCreate(&ev0) == hipSuccess) (void)hipEventRecord(ev0, st);
  }
  // Ends the interval early (before a host synchronisation of the call).
  void stop() {
    hipEvent_t ev1 = nullptr;
    if (ev0 && hipEventCreate(&ev1) == hipSuccess && hipEventRecord(ev1, st) == hipSuccess)
      timing_push(kind, ev0, ev1);
    else if (ev0)
      (void)hipEventDestroy(ev0);
    ev0 = nullptr;
  }
  ~TimedScope() { stop(); }
  TimedScope(const TimedScope&) = delete;
  TimedScope& operator=(const TimedScope&) = delete;
};

// ---------------------------------------------------------------- keys
// A voxel key is the triple floor(x / v) per axis; keys are limited to
// [-2^20, 2^20) and packed as three 21-bit fields biased by 2^20 into the low
// 63 bits of a uint64.  The all-ones word marks an empty hash slot and sorts
// after every key (used for non-finite points).
constexpr int64_t kKeyBias = int64_t(1) << 20;
constexpr uint64_t kEmptyKey = ~uint64_t(0);
constexpr int kKeyBits = 63;

__host__ __device__ inline uint64_t pack_key(int64_t kx, int64_t ky, int64_t kz) {
  return (uint64_t(kx + kKeyBias) << 42) | (uint64_t(ky + kKeyBias) << 21) |
         uint64_t(kz + kKeyBias);
}
__host__ __device__ inline bool key_ok(int64_t k) { return k >= -kKeyBias && k < kKeyBias; }
__host__ __device__ inline int64_t key_x(uint64_t k) { return int64_t((k >> 42) & 0x1FFFFF) - kKeyBias; }
__host__ __device__ inline int64_t key_y(uint64_t k) { return int64_t((k >> 21) & 0x1FFFFF) - kKeyBias; }
__host__ __device__ inline int64_t key_z(uint64_t k) { return int64_t(k & 0x1FFFFF) - kKeyBias; }

// Spatial hash of Teschner et al. as used by Niessner et al. (the hash the
// paper's voxel map employs): XOR of the three indices times large primes,
// folded to the power-of-two table by Fibonacci hashing of the 32-bit result.
__host__ __device__ inline uint32_t voxel_hash(int64_t kx, int64_t ky, int64_t kz,
                                               int log2_slots) {
  uint32_t h = (uint32_t(kx) * 73856093u) ^ (uint32_t(ky) * 19349669u) ^
               (uint32_t(kz) * 83492791u);
  return uint32_t((uint64_t(h) * 0x9E3779B97F4A7C15ull) >> (64 - log2_slots));
}

struct alignas(16) Slot {
  uint64_t key;   // kEmptyKey when free
  int32_t vox;    // compact voxel index
  int32_t aux;    // map: points the voxel holds (mirror of vox_count), so one
                  // 16-byte probe yields key, voxel and count; scan grid: scan id
};

// A slot in one memory round trip.  Read field by field (or even as one
// 16-byte vector), the compiler fetches the key, compares it and only then
// fetches voxel and count; the empty asm statement takes those two words
// where the load is, so all four arrive together.
__device__ inline Slot load_slot(const Slot* p) {
  const uint4 w = *reinterpret_cast<const uint4*>(p);
  uint32_t vox = w.z, aux = w.w;
  asm volatile("" : "+v"(vox), "+v"(aux));
  Slot s;
  s.key = uint64_t(w.x) | (uint64_t(w.y) << 32);
  s.vox = int32_t(vox);
  s.aux = int32_t(aux);
  return s;
}

// Nearest-neighbour certificate of a map point, stored per slot of vox_pts
// (voxel-major, so the certificates a search reads lie next to the points it
// reads): the point's own coordinates and rho, then its kCertK nearest other
// map points within v, each as (x, y, z, vox_pts slot bits) (slot -1 past
// the last), so that a certificate reads one 128-byte row and no point by
// its slot.  rho is at most half the distance from the point to every map
// point not in that list (v/2 when fewer than kCertK + 1 others lie within
// v), rounded down.  A query x whose distance to the point q is below rho is
// farther than that from every unlisted point (triangle inequality:
// |x - q''| >= |q - q''| - |x - q| >= 2 rho - |x - q| > |x - q|), so q is x's
// nearest map point once it also ranks before every listed point.  A row
// stays valid while the listed slots keep their points: an insert only adds
// points to free slots (the rows of the points within v of an added point are
// rebuilt) and an eviction, which moves points, rebuilds every row.
constexpr int kCertK = 7;
struct alignas(128) CertRow {
  float x, y, z, rho;
  float4 nbr[kCertK];
};

// Device view of a map, passed by value to kernels.
struct MapView {
  const Slot* slots;
  const int32_t* vox_count;     // [voxel_cap]
  const float4* vox_pts;        // [voxel_cap * nmax]: x, y, z, id (int bits)
  const float4* cov;            // [point_cap * 2]: (xx,xy,xz,yy), (yz,zz,valid,0)
  const float4* vox_cov;        // [voxel_cap * nmax * 2]: the same records by vox_pts slot
  const uint32_t* vox_nbr;      // [voxel_cap * 26]: neighbour voxel << 7 | its count
  const float* pt_xyz;          // [3][point_cap]
  const CertRow* cert;          // [voxel_cap * nmax], by vox_pts slot
  // ghost voxels: the empty voxels next to an occupied one, each with a
  // neighbour-table row like an occupied voxel's (ghost_ok: the table holds
  // every such voxel, else searches probe the neighbours one by one)
  const Slot* gslots;           // key, vox = ghost index
  const uint32_t* gnbr;         // [ghost_cap * 26]
  uint32_t gmask;
  int32_t glog2;
  int32_t ghost_ok;
  int64_t point_cap;
  double v;
  int32_t nmax;
  int32_t log2_slots;
  uint32_t slot_mask;
  // fine search index (cells of v/2): points sorted by cell, cell -> run
  const float4* fine_pts;     // [n_points]: x, y, z, id bits
  const Slot* fine_slots;     // key, vox = run start, aux = run length
  uint32_t fine_mask;
  int32_t fine_log2;
  int32_t fine_ok;            // index built for the current map contents
  double fc;                  // fine cell edge (v / 2, a power of two)
  double inv_fc;
};

// Neighbour table of the map: for every voxel and each of its 26 neighbour
// directions (code = (ox+1)*9 + (oy+1)*3 + (oz+1), code 13 = the voxel
// itself left out), the neighbour's voxel index << 7 | its point count, or
// kNbrNone when the neighbour voxel does not exist.
constexpr uint32_t kNbrNone = 0xFFFFFFFFu;
constexpr int kNbrCountBits = 7;
__host__ __device__ inline int nbr_dir(int code) { return code < 13 ? code : code - 1; }

// Ghost index of empty voxel (kx, ky, kz) next to the map, or -1.
__device__ inline int32_t ghost_find(const MapView& m, int64_t kx, int64_t ky, int64_t kz) {
  if (!key_ok(kx) || !key_ok(ky) || !key_ok(kz)) return -1;
  const uint64_t key = pack_key(kx, ky, kz);
  uint32_t s = voxel_hash(kx, ky, kz, m.glog2);
  for (uint32_t probe = 0; probe <= m.gmask; ++probe) {
    const Slot sl = load_slot(&m.gslots[s]);
    if (sl.key == key) return sl.vox;
    if (sl.key == kEmptyKey) return -1;
    s = (s + 1) & m.gmask;
  }
  return -1;
}

// Run [start, start + *cnt) of fine cell (kx, ky, kz) in fine_pts, or -1.
__device__ inline int32_t fine_find(const MapView& m, int64_t kx, int64_t ky, int64_t kz,
                                    int32_t* cnt) {
  *cnt = 0;
  if (!key_ok(kx) || !key_ok(ky) || !key_ok(kz)) return -1;
  const uint64_t key = pack_key(kx, ky, kz);
  uint32_t s = voxel_hash(kx, ky, kz, m.fine_log2);
  for (uint32_t probe = 0; probe <= m.fine_mask; ++probe) {
    const Slot sl = load_slot(&m.fine_slots[s]);
    if (sl.key == key) {
      *cnt = sl.aux;
      return sl.vox;
    }
    if (sl.key == kEmptyKey) return -1;
    s = (s + 1) & m.fine_mask;
  }
  return -1;
}

// Voxel index of key (kx, ky, kz), or -1; *cnt receives its point count (0
// when absent).
__device__ inline int32_t map_find(const MapView& m, int64_t kx, int64_t ky, int64_t kz,
                                   int32_t* cnt) {
  *cnt = 0;
  if (!key_ok(kx) || !key_ok(ky) || !key_ok(kz)) return -1;
  uint64_t key = pack_key(kx, ky, kz);
  uint32_t s = voxel_hash(kx, ky, kz, m.log2_slots);
  for (uint32_t probe = 0; probe <= m.slot_mask; ++probe) {
    const Slot sl = load_slot(&m.slots[s]);
    if (sl.key == key) {
      *cnt = sl.aux;
      return sl.vox;
    }
    if (sl.key == kEmptyKey) return -1;
    s = (s + 1) & m.slot_mask;
  }
  return -1;
}

// FP64 squared distance, fixed evaluation order, no contraction (the library
// is compiled with -ffp-contract=off).
__host__ __device__ inline double dist2(double ax, double ay, double az, double bx,
                                        double by, double bz) {
  double dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

// (d2, id) lexicographic order used by every ranking.
__host__ __device__ inline bool rank_less(double da, int32_t ia, double db, int32_t ib) {
  return da < db || (da == db && ia < ib);
}

// Conservative squared lower bound of the distance from q to any point of the
// voxel at offset (ox, oy, oz) from q's voxel (kq).  A slack of 1e-7 v per
// axis absorbs every rounding of the key and distance arithmetic, so a voxel
// is skipped only when none of its points could rank.
__device__ inline double voxel_lb2(double qx, double qy, double qz, int64_t kqx,
                                   int64_t kqy, int64_t kqz, int ox, int oy, int oz,
                                   double v) {
  double slack = 1e-7 * v;
  double g, s = 0.0;
  if (ox < 0) { g = qx - double(kqx) * v - slack; s += g > 0 ? g * g : 0.0; }
  if (ox > 0) { g = double(kqx + 1) * v - qx - slack; s += g > 0 ? g * g : 0.0; }
  if (oy < 0) { g = qy - double(kqy) * v - slack; s += g > 0 ? g * g : 0.0; }
  if (oy > 0) { g = double(kqy + 1) * v - qy - slack; s += g > 0 ? g * g : 0.0; }
  if (oz < 0) { g = qz - double(kqz) * v - slack; s += g > 0 ? g * g : 0.0; }
  if (oz > 0) { g = double(kqz + 1) * v - qz - slack; s += g > 0 ? g * g : 0.0; }
  return s;
}

// The 27 neighbour offsets, own voxel first, then the 6 faces, 12 edges and
// 8 corners (increasing minimum distance), encoded as (ox+1)*9+(oy+1)*3+(oz+1).
static __constant__ int8_t kNbrOrder[27] = {13, 4, 22, 10, 16, 12, 14, 1,  3,  5,
                                            7,  9, 11, 15, 17, 19, 21, 23, 25, 0,
                                            2,  6,  8, 18, 20, 24, 26};

// ---------------------------------------------------------------- scratch
// The stream-ordered pool of the current device that scratch comes from: one
// per device, created on first use, keeping freed memory for later calls.
far_status_t scratch_pool(hipMemPool_t* out);

// Stream-ordered device scratch, freed when the guard leaves scope.  Pieces
// are cut from chunks of at least kScratchChunk bytes taken from the pool,
// so a call with many temporary buffers makes a few pool requests (each
// costs microseconds of host time) instead of one per buffer.
// With an arena (a preallocated device buffer) it hands out 256-byte aligned
// pieces of it instead, which is what code recorded into a graph needs.
constexpr size_t kScratchChunk = size_t(64) << 20;

struct Scratch {
  hipStream_t stream;
  std::vector<void*> ptrs;
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  char* chunk = nullptr;
  size_t chunk_cap = 0, chunk_used = 0;
  explicit Scratch(hipStream_t s) : stream(s) {}
  Scratch(hipStream_t s, void* buf, size_t cap)
      : stream(s), arena(static_cast<char*>(buf)), arena_cap(cap) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, stream);
  }
  template <class T>
  far_status_t get(T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    size_t bytes = count * sizeof(T);
    if (arena) {
      size_t at = (arena_used + 255) & ~size_t(255);
      if (at + bytes > arena_cap) {
        set_error("internal: scratch arena of %zu bytes exhausted", arena_cap);
        return FAR_E_CAPACITY;
      }
      arena_used = at + bytes;
      *out = reinterpret_cast<T*>(arena + at);
      return FAR_OK;
    }
    const size_t at = (chunk_used + 255) & ~size_t(255);
    if (chunk && at + bytes <= chunk_cap) {
      chunk_used = at + bytes;
      *out = reinterpret_cast<T*>(chunk + at);
      return FAR_OK;
    }
    hipMemPool_t pool;
    FAR_TRY(scratch_pool(&pool));
    const size_t cap = bytes > kScratchChunk ? bytes : kScratchChunk;
    void* p = nullptr;
    FAR_HIP(hipMallocFromPoolAsync(&p, cap, pool, stream));
    ptrs.push_back(p);
    chunk = static_cast<char*>(p);
    chunk_cap = cap;
    chunk_used = bytes;
    *out = static_cast<T*>(p);
    return FAR_OK;
  }
};

// Upper bound of the scratch bytes radix_sort_pairs takes for n elements.
inline size_t radix_sort_scratch_bytes(int64_t n) {
  size_t nb = size_t((n + 4095) / 4096) + 1;
  size_t hist = 256 * nb * 4 + 256;
  size_t sums = 0, m = 256 * nb;
  for (int lvl = 0; lvl < 4; ++lvl) {
    m = (m + 2047) / 2048;
    sums += m * 4 + 256;
  }
  return hist + 8 * sums + 4096;
}

// ---------------------------------------------------------------- primitives
// Stable LSD radix sort of (key, value) pairs by key bits [0, bits); the
// *_alt buffers are scratch of the same size.  With in_alt NULL the result
// lands in keys/vals; otherwise it stays in whichever pair the last pass
// wrote and *in_alt says whether that is the *_alt pair (no copy is made).
far_status_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                              uint32_t* vals_alt, int64_t n, int bits, hipStream_t st,
                              Scratch& scr, bool* in_alt = nullptr);
// Exclusive prefix sum of n uint32 values; the total goes to *total [dev]
// when total is not NULL.  in and out may alias.
far_status_t scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                            hipStream_t st, Scratch& scr);

// ---------------------------------------------------------------- covariances
// Regularised covariances of the map points with ids [id0, id1) on the map.
far_status_t map_covariances(const MapView& m, float4* cov_out, int64_t id0, int64_t id1,
                             int32_t k, hipStream_t st);

int device_cu_count();

// Align workspace owned by a map (defined with the GICP kernels).
struct AlignWS;
void free_ws(AlignWS* w);

}  // namespace far

// Host-side map object.
struct far_map_s {
  far_map_params_t p;
  int32_t sched_tile = 256;   // linearisation tile (points per block)
  int32_t sched_fine = 0;     // correspondence search over the fine index
  double dmin;
  int64_t slots;
  int log2_slots;
  int64_t voxel_cap;
  far::Slot* slots_d = nullptr;
  int32_t* vox_count = nullptr;
  uint64_t* vox_key = nullptr;
  float4* vox_pts = nullptr;
  float4* cov = nullptr;
  float4* vox_cov = nullptr;
  uint32_t* vox_nbr = nullptr;
  float* pt_xyz = nullptr;
  int32_t* pt_loc = nullptr;
  int32_t* vox_slot = nullptr;
  // nearest-neighbour certificates (by vox_pts slot) and the per-voxel marks
  // of the voxels whose points' certificates an insert recomputes
  far::CertRow* cert = nullptr;
  uint32_t* cert_mark = nullptr;
  uint32_t cert_gen = 0;
  // ghost voxels (empty voxels next to an occupied one): hash table, keys
  // and neighbour rows by ghost index, the device count of ghosts claimed
  far::Slot* gslots = nullptr;
  uint64_t* gkey = nullptr;
  uint32_t* gnbr = nullptr;
  uint32_t* gcount = nullptr;
  int64_t ghost_cap = 0;
  int64_t gslots_n = 0;
  int glog2 = 0;
  int64_t n_ghosts = 0;         // as of the last map update (host copy)
  bool ghost_ok = true;
  // fine search index, rebuilt lazily after the map changes
  float4* fine_pts = nullptr;
  far::Slot* fine_slots = nullptr;
  int64_t fine_nslots = 0;
  int fine_log2 = 0;
  bool fine_ok = false;
  int64_t n_points = 0;
  int64_t n_voxels = 0;
  int device = 0;
  int64_t bytes = 0;
  far::AlignWS* ws = nullptr;
  far::MapView view() const {
    far::MapView m;
    m.slots = slots_d;
    m.vox_count = vox_count;
    m.vox_pts = vox_pts;
    m.cov = cov;
    m.vox_cov = vox_cov;
    m.vox_nbr = vox_nbr;
    m.pt_xyz = pt_xyz;
    m.cert = cert;
    m.gslots = gslots;
    m.gnbr = gnbr;
    m.gmask = uint32_t(gslots_n - 1);
    m.glog2 = glog2;
    m.ghost_ok = ghost_ok ? 1 : 0;
    m.point_cap = p.point_capacity;
    m.v = p.voxel_size;
    m.nmax = p.max_pts_per_voxel;
    m.log2_slots = log2_slots;
    m.slot_mask = uint32_t(slots - 1);
    m.fine_pts = fine_pts;
    m.fine_slots = fine_slots;
    m.fine_mask = uint32_t(fine_nslots - 1);
    m.fine_log2 = fine_log2;
    m.fine_ok = fine_ok ? 1 : 0;
    m.fc = 0.5 * p.voxel_size;
    m.inv_fc = 1.0 / m.fc;
    return m;
  }
};

namespace far {
// Build the fine search index of the map if it is stale (stream-ordered;
// no-op when the voxel edge is not a power of two or a point lies outside
// the fine key range, in which case searches use the voxels).
far_status_t fine_build(far_map_s* m, hipStream_t st);
}  // namespace far
