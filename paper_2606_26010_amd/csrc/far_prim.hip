// far_prim.hip -- device-wide primitives: stable LSD radix sort of (uint64 key,
// uint32 value) pairs and an exclusive prefix sum, written for wave64.
//
// The insert needs a *stable* grouping of points by voxel key so that each
// voxel's candidates are visited in input order (the sequential capped-insert
// semantics); an LSD radix sort whose every pass is stable gives exactly that.
#include <mutex>
#include <utility>
#include <vector>

#include "far_internal.h"

namespace far {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// ---------------------------------------------------------------- scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and writes the block total.
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    uint32_t s = lds[w];
    pre += (w < wave) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_tile_sums(const uint32_t* in, int64_t n,
                                                             uint32_t* sums) {
  __shared__ uint32_t lds[kWaves];
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) s += (base + j < n) ? in[base + j] : 0u;
  uint32_t tot;
  (void)block_exscan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan each tile, adding carry[blockIdx.x] (scanned tile sums) when given.
// The last tile writes the grand total.
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const uint32_t* in, uint32_t* out,
                                                         int64_t n, const uint32_t* carry,
                                                         uint32_t* total) {
  __shared__ uint32_t lds[kWaves];
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0u;
    s += v[j];
  }
  uint32_t tot;
  uint32_t pre = block_exscan(s, lds, &tot);
  uint32_t c = carry ? carry[blockIdx.x] : 0u;
  uint32_t run = c + pre;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = c + tot;
}

// ---------------------------------------------------------------- radix sort
constexpr int kSortItems = 16;
constexpr int kSortTile = kThreads * kSortItems;

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t* keys, int64_t n,
                                                      int shift, uint32_t* hist,
                                                      int64_t nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = int64_t(blockIdx.x) * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + int64_t(r) * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[uint32_t(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one 8-bit digit.  Each block ranks its tile in LDS, then
// writes it out digit by digit, so that equal digits of a tile land in
// consecutive addresses (whole cache lines) instead of one scattered element
// per lane.  Each wave ranks its own contiguous quarter of the tile in index
// order, 64 elements a round: an element's rank among equal digits is the
// wave's running count of its digit plus its equal digits in lower lanes
// (found with eight ballots); one prefix over the waves per digit then
// places the quarters after each other.  hist holds the exclusive prefix,
// digit-major, of the per-block digit counts, so a block's count of digit d
// is the difference of its entry and the next one (n after the last).
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint64_t* kin,
                                                         const uint32_t* vin, uint64_t* kout,
                                                         uint32_t* vout, int64_t n, int shift,
                                                         const uint32_t* hist,
                                                         int64_t nblocks) {
  constexpr int kPerWave = kSortTile / kWaves;
  constexpr int kRounds = kPerWave / 64;
  __shared__ uint64_t lkey[kSortTile];
  __shared__ uint32_t lval[kSortTile];
  __shared__ uint32_t gbase[256];   // global start of this block's digit d
  __shared__ uint32_t lbase[256];   // local start of digit d in the tile
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t wsum[kWaves];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t blk = int64_t(blockIdx.x) * kSortTile;
  const int64_t wbase = blk + int64_t(wave) * kPerWave;
  // the wave's quarter into registers first, so that ranking does not wait
  uint64_t kr[kRounds];
  uint32_t vr[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    kr[r] = i < n ? kin[i] : 0ull;
    vr[r] = i < n ? vin[i] : 0u;
  }
  const int64_t hi = int64_t(t) * nblocks + blockIdx.x;
  const uint32_t g0 = hist[hi];
  const uint32_t cnt = (hi + 1 < 256 * nblocks ? hist[hi + 1] : uint32_t(n)) - g0;
  gbase[t] = g0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  // exclusive prefix of the 256 counts: within each wave, then across waves
  uint32_t incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  lbase[t] = before + incl - cnt;
  // rank inside the wave's quarter (the wave's LDS operations stay in order,
  // so a group's leader updates the count after every lane of it has read it)
  const uint64_t lower = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t pos[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool ok = wbase + r * 64 + lane < n;
    const uint32_t d = uint32_t(kr[r] >> shift) & 255u;
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      m &= bit ? bal : ~bal;
    }
    const uint32_t rank = __popcll(m & lower);
    const uint32_t prev = wcnt[wave][d];
    pos[r] = prev + rank;
    if (ok && rank == 0) wcnt[wave][d] = prev + __popcll(m);
  }
  __syncthreads();
  // per digit, the waves' quarters one after the other from the digit's start
  uint32_t run = lbase[t];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t c = wcnt[w][t];
    wcnt[w][t] = run;
    run += c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
    if (wbase + r * 64 + lane < n) {
      const uint32_t off = wcnt[wave][uint32_t(kr[r] >> shift) & 255u] + pos[r];
      lkey[off] = kr[r];
      lval[off] = vr[r];
    }
  __syncthreads();
  // write out in local order: consecutive positions of one digit go to
  // consecutive global addresses
  const int tile = int(min(int64_t(kSortTile), n - blk));
  for (int p = t; p < tile; p += kThreads) {
    const uint64_t k = lkey[p];
    const uint32_t d = uint32_t(k >> shift) & 255u;
    const uint32_t off = gbase[d] + uint32_t(p) - lbase[d];
    kout[off] = k;
    vout[off] = lval[p];
  }
}

}  // namespace

far_status_t scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                            hipStream_t st, Scratch& scr) {
  if (n <= 0) {
    if (total) FAR_HIP(hipMemsetAsync(total, 0, sizeof(uint32_t), st));
    return FAR_OK;
  }
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    k_scan_tiles<<<1, kThreads, 0, st>>>(in, out, n, nullptr, total);
    FAR_HIP(hipGetLastError());
    return FAR_OK;
  }
  uint32_t* sums = nullptr;
  FAR_TRY(scr.get(&sums, size_t(tiles)));
  k_scan_tile_sums<<<dim3(uint32_t(tiles)), kThreads, 0, st>>>(in, n, sums);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(sums, sums, tiles, nullptr, st, scr));
  k_scan_tiles<<<dim3(uint32_t(tiles)), kThreads, 0, st>>>(in, out, n, sums, total);
  FAR_HIP(hipGetLastError());
  return FAR_OK;
}

far_status_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                              uint32_t* vals_alt, int64_t n, int bits, hipStream_t st,
                              Scratch& scr, bool* in_alt) {
  if (in_alt) *in_alt = false;
  if (n <= 1 || bits <= 0) return FAR_OK;
  int64_t nblocks = (n + kSortTile - 1) / kSortTile;
  uint32_t* hist = nullptr;
  FAR_TRY(scr.get(&hist, size_t(256 * nblocks)));
  uint64_t *ka = keys, *kb = keys_alt;
  uint32_t *va = vals, *vb = vals_alt;
  int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    k_rs_hist<<<dim3(uint32_t(nblocks)), kThreads, 0, st>>>(ka, n, shift, hist, nblocks);
    FAR_HIP(hipGetLastError());
    FAR_TRY(scan_exclusive(hist, hist, 256 * nblocks, nullptr, st, scr));
    k_rs_scatter<<<dim3(uint32_t(nblocks)), kThreads, 0, st>>>(ka, va, kb, vb, n, shift,
                                                               hist, nblocks);
    FAR_HIP(hipGetLastError());
    uint64_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  if (in_alt) {
    *in_alt = ka != keys;
    return FAR_OK;
  }
  if (ka != keys) {
    FAR_HIP(hipMemcpyAsync(keys, ka, size_t(n) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    FAR_HIP(hipMemcpyAsync(vals, va, size_t(n) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
  return FAR_OK;
}

// ---------------------------------------------------------------- scratch pool
// A call's temporary buffers are allocated and freed on its stream.  The
// device's default pool hands freed memory back to the driver at every
// synchronisation (release threshold 0), so each call would map its scratch
// afresh, which costs more than many of the kernels it serves.  The library's
// own pool keeps what it has reserved (threshold unlimited) until
// far_scratch_release: its footprint is the largest scratch any one call
// has needed, far below the device memory of the workloads it serves.
namespace {
struct Pools {
  std::mutex mu;
  std::vector<hipMemPool_t> pool;   // per device id, null until first use
};
Pools& pools() {
  static Pools p;
  return p;
}
}  // namespace

far_status_t scratch_pool(hipMemPool_t* out) {
  *out = nullptr;
  int dev = 0;
  FAR_HIP(hipGetDevice(&dev));
  Pools& P = pools();
  std::lock_guard<std::mutex> lk(P.mu);
  if (size_t(dev) >= P.pool.size()) P.pool.resize(size_t(dev) + 1, nullptr);
  if (!P.pool[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t p = nullptr;
    FAR_HIP(hipMemPoolCreate(&p, &props));
    uint64_t keep = ~uint64_t(0);
    const hipError_t e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(p);
      return hip_fail(e, "hipMemPoolSetAttribute(release threshold)", __FILE__, __LINE__);
    }
    P.pool[dev] = p;
  }
  *out = P.pool[dev];
  return FAR_OK;
}

// ---------------------------------------------------------------- timing
namespace {
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[FAR_TIME_KINDS];
  double ms[FAR_TIME_KINDS] = {};
  int64_t count[FAR_TIME_KINDS] = {};
};
Timing& timing() {
  static Timing t;
  return t;
}
}  // namespace

bool timing_on() {
  std::lock_guard<std::mutex> lk(timing().mu);
  return timing().on;
}

void timing_push(int kind, hipEvent_t ev0, hipEvent_t ev1) {
  std::lock_guard<std::mutex> lk(timing().mu);
  timing().pending[kind].push_back({ev0, ev1});
}

}  // namespace far

extern "C" {

far_status_t far_scratch_release(void) {
  far::Pools& P = far::pools();
  std::lock_guard<std::mutex> lk(P.mu);
  for (hipMemPool_t p : P.pool)
    if (p) FAR_HIP(hipMemPoolTrimTo(p, 0));
  return FAR_OK;
}

far_status_t far_scratch_reserved(int64_t* bytes) {
  if (!bytes) {
    far::set_error("far_scratch_reserved: invalid argument");
    return FAR_E_INVALID;
  }
  *bytes = 0;
  int dev = 0;
  FAR_HIP(hipGetDevice(&dev));
  far::Pools& P = far::pools();
  std::lock_guard<std::mutex> lk(P.mu);
  if (size_t(dev) >= P.pool.size() || !P.pool[dev]) return FAR_OK;
  uint64_t v = 0;
  FAR_HIP(hipMemPoolGetAttribute(P.pool[dev], hipMemPoolAttrReservedMemCurrent, &v));
  *bytes = int64_t(v);
  return FAR_OK;
}

far_status_t far_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(far::timing().mu);
  far::timing().on = on != 0;
  return FAR_OK;
}

far_status_t far_timing_read_kind(int32_t kind, double* ms, int64_t* count, int32_t reset) {
  if (kind < 0 || kind >= FAR_TIME_KINDS) {
    far::set_error("far_timing_read_kind: kind %d out of range", kind);
    return FAR_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(far::timing().mu);
  far::Timing& t = far::timing();
  for (auto& pr : t.pending[kind]) {
    FAR_HIP(hipEventSynchronize(pr.second));
    float e = 0.0f;
    FAR_HIP(hipEventElapsedTime(&e, pr.first, pr.second));
    t.ms[kind] += e;
    t.count[kind] += 1;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  t.pending[kind].clear();
  if (ms) *ms = t.ms[kind];
  if (count) *count = t.count[kind];
  if (reset) {
    t.ms[kind] = 0.0;
    t.count[kind] = 0;
  }
  return FAR_OK;
}

far_status_t far_timing_read(double* linearize_ms, int64_t* launches, int32_t reset) {
  return far_timing_read_kind(FAR_TIME_LINEARIZE, linearize_ms, launches, reset);
}

}  // extern "C"
