// far_map.hip -- the voxel hash map (Sec. III-A.2 cuVoxelMap paragraph,
// Sec. III-A.3 Adaptive, Local Submap): create, capped insert with the
// covariances of the added points, k-nearest-neighbour query, export, stats,
// and the covariances of a scan against its own (uncapped) voxel grid.
//
// Layout in HBM (all fixed at create):
//   slots     Slot[S]            open addressing, linear probing step 1,
//                                S = 2^ceil(log2(2 * voxel_capacity))
//   vox_count int32[Vc]          points held per voxel
//   vox_key   uint64[Vc]         packed key per voxel
//   vox_pts   float4[Vc * Nmax]  voxel-major point store: x, y, z, id bits
//   cov       float4[Pc * 2]     per id: (xx, xy, xz, yy), (yz, zz, valid, 0)
//   pt_xyz    float[3][Pc]       per id coordinates (SoA)
//   pt_loc    int32[Pc]          per id slot in vox_pts
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <type_traits>

#include <algorithm>

#include "far_knn.h"

namespace far {

// ---------------------------------------------------------------- errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

far_status_t hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("HIP error %d (%s) in %s at %s:%d", int(e), hipGetErrorString(e), what, file, line);
  return FAR_E_HIP;
}

int device_cu_count() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    cus[dev] = prop.multiProcessorCount;
  }
  return cus[dev];
}

namespace {

constexpr int kT = 256;

inline unsigned blocks_for(int64_t n, int per = kT) {
  int64_t b = (n + per - 1) / per;
  return unsigned(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------- keys
// Voxel key of every point (Sec. III-A.2: the key is the voxel's 3-D index).
// Non-finite points get the empty key (they sort last and are skipped);
// out-of-range points are counted and make the call fail.
__global__ __launch_bounds__(kT) void k_keys(const float* xyz, int64_t n, double v,
                                             uint64_t* keys, uint32_t* vals,
                                             uint32_t* counters) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  uint64_t key = kEmptyKey;
  if (isfinite(x) && isfinite(y) && isfinite(z)) {
    int64_t kx, ky, kz;
    if (voxel_index(double(x), v, &kx) && voxel_index(double(y), v, &ky) &&
        voxel_index(double(z), v, &kz))
      key = pack_key(kx, ky, kz);
    else
      atomicAdd(&counters[1], 1u);
  } else {
    atomicAdd(&counters[0], 1u);
  }
  keys[i] = key;
  vals[i] = uint32_t(i);
}

// Segment heads of the sorted keys (first element of each run of equal keys).
__global__ __launch_bounds__(kT) void k_heads(const uint64_t* keys, int64_t n,
                                              uint32_t* head) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  uint64_t k = keys[j];
  head[j] = (k != kEmptyKey && (j == 0 || keys[j - 1] != k)) ? 1u : 0u;
}

// ---------------------------------------------------------------- downsample
// Keep flags of the first point (in input order) of every voxel: after the
// stable sort every input index appears once in vals and a run's head holds
// its smallest index, so writing head[j] to flag[vals[j]] sets every flag.
__global__ __launch_bounds__(kT) void k_ds_flags(const uint32_t* vals, const uint32_t* head,
                                                 int64_t n, uint32_t* flag) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  flag[vals[j]] = head[j];
}

// Compaction of the kept points in input order, SoA with row stride n_out.
__global__ __launch_bounds__(kT) void k_ds_scatter(const float* xyz, int64_t n,
                                                   const uint32_t* flag, const uint32_t* pos,
                                                   int64_t n_out, float* out, int32_t* keep) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n || !flag[i]) return;
  int64_t o = pos[i];
  out[o] = xyz[i];
  out[n_out + o] = xyz[n + i];
  out[2 * n_out + o] = xyz[2 * n + i];
  if (keep) keep[o] = int32_t(i);
}

// ---------------------------------------------------------------- transform
struct Rigid {
  double r[12];  // rows of [R | t]
};

// out = R s + t per point, FP64 in the order ((R_r0 x + R_r1 y) + R_r2 z) + t_r
// (no contraction: the file is built with -ffp-contract=off), rounded to float.
// Every thread reads its point before writing it, so out may alias xyz.
__global__ __launch_bounds__(kT) void k_transform(const float* xyz, int64_t n, Rigid T,
                                                  float* out) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  float o[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    o[r] = float(((T.r[4 * r] * x + T.r[4 * r + 1] * y) + T.r[4 * r + 2] * z) + T.r[4 * r + 3]);
  out[i] = o[0];
  out[n + i] = o[1];
  out[2 * n + i] = o[2];
}

// Segment bounds: seg_start[s] and seg_end[s] for every run s.
__global__ __launch_bounds__(kT) void k_seg_bounds(const uint64_t* keys, int64_t n,
                                                   const uint32_t* head,
                                                   const uint32_t* head_scan,
                                                   uint32_t* seg_start, uint32_t* seg_end) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  uint64_t k = keys[j];
  if (k == kEmptyKey) return;
  uint32_t s = head_scan[j] + head[j] - 1;
  if (head[j]) seg_start[s] = uint32_t(j);
  if (j == n - 1 || keys[j + 1] != k) seg_end[s] = uint32_t(j + 1);
}

// Look each run's key up in the table; flag runs whose voxel is new.
__global__ __launch_bounds__(kT) void k_seg_lookup(MapView m, const uint64_t* keys,
                                                   const uint32_t* seg_start,
                                                   const uint32_t* n_seg, int64_t n,
                                                   int32_t* seg_vox, uint32_t* is_new) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n) return;
  if (s >= int64_t(*n_seg)) {
    is_new[s] = 0;
    return;
  }
  uint64_t key = keys[seg_start[s]];
  int32_t cnt;
  int32_t vox = map_find(m, key_x(key), key_y(key), key_z(key), &cnt);
  seg_vox[s] = vox;
  is_new[s] = vox < 0 ? 1u : 0u;
}

// Claim a slot for every new voxel; new voxels are numbered in sorted key
// order after the existing ones, so the layout is deterministic.
__global__ __launch_bounds__(kT) void k_seg_claim(Slot* slots, uint32_t slot_mask,
                                                  int log2_slots, const uint64_t* keys,
                                                  const uint32_t* seg_start,
                                                  const uint32_t* is_new,
                                                  const uint32_t* new_rank, int64_t n_seg,
                                                  int64_t n_vox_old, int32_t* seg_vox,
                                                  uint64_t* vox_key, int32_t* vox_slot) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg || !is_new[s]) return;
  uint64_t key = keys[seg_start[s]];
  int32_t vox = int32_t(n_vox_old + new_rank[s]);
  uint32_t h = voxel_hash(key_x(key), key_y(key), key_z(key), log2_slots);
  for (uint32_t probe = 0; probe <= slot_mask; ++probe) {
    unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&slots[h].key),
                                       (unsigned long long)kEmptyKey,
                                       (unsigned long long)key);
    if (old == kEmptyKey) {
      slots[h].vox = vox;
      slots[h].aux = 0;
      vox_slot[vox] = int32_t(h);
      break;
    }
    h = (h + 1) & slot_mask;
  }
  seg_vox[s] = vox;
  vox_key[vox] = key;
}

// Sequential capped insert of one voxel's candidates in input order (one
// thread per voxel run; runs are stable-sorted so candidates appear in input
// order).  A candidate is accepted while the voxel holds fewer than its cap
// and, with spacing on, it is at least dmin from every point already there.
// Accepted points are appended to the voxel's store right away, so later
// candidates of the same run are checked against them.
__global__ __launch_bounds__(kT) void k_greedy(const float* xyz, int64_t n,
                                               const int32_t* caps, int32_t nmax,
                                               double dmin2, const uint32_t* vals,
                                               const uint32_t* seg_start,
                                               const uint32_t* seg_end, int64_t n_seg,
                                               const int32_t* seg_vox,
                                               const int32_t* vox_count, float4* vox_pts,
                                               uint32_t* acc_flag, int32_t* acc_pos,
                                               int32_t* seg_newcount) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  int32_t vox = seg_vox[s];
  int32_t cnt = vox_count[vox];
  float4* store = vox_pts + int64_t(vox) * nmax;
  for (uint32_t j = seg_start[s]; j < seg_end[s]; ++j) {
    uint32_t i = vals[j];
    int32_t cap = caps ? min(caps[i], nmax) : nmax;
    if (cnt >= cap) continue;
    float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    bool ok = true;
    if (dmin2 > 0.0) {
      for (int32_t q = 0; q < cnt; ++q) {
        float4 p = store[q];
        if (dist2(double(x), double(y), double(z), double(p.x), double(p.y), double(p.z)) <
            dmin2) {
          ok = false;
          break;
        }
      }
    }
    if (!ok) continue;
    store[cnt] = make_float4(x, y, z, __int_as_float(-1));
    acc_flag[i] = 1u;
    acc_pos[i] = int32_t(int64_t(vox) * nmax + cnt);
    ++cnt;
  }
  seg_newcount[s] = cnt;
}

// Give accepted points their ids (input order) and record them by id.
__global__ __launch_bounds__(kT) void k_commit(const float* xyz, int64_t n,
                                               const uint32_t* acc_flag,
                                               const uint32_t* id_local,
                                               const int32_t* acc_pos, int64_t id0,
                                               int64_t point_cap, float4* vox_pts,
                                               float* pt_xyz, int32_t* pt_loc) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n || !acc_flag[i]) return;
  int64_t id = id0 + id_local[i];
  if (id >= point_cap) return;
  int32_t pos = acc_pos[i];
  vox_pts[pos].w = __int_as_float(int32_t(id));
  pt_xyz[id] = xyz[i];
  pt_xyz[point_cap + id] = xyz[n + i];
  pt_xyz[2 * point_cap + id] = xyz[2 * n + i];
  pt_loc[id] = pos;
}

// New per-voxel counts.  When the point capacity truncated the batch, only
// the accepted prefix whose ids fit is kept.
__global__ __launch_bounds__(kT) void k_counts(int64_t n_seg, const int32_t* seg_vox,
                                               const int32_t* seg_newcount, bool truncated,
                                               const uint32_t* vals, const uint32_t* seg_start,
                                               const uint32_t* seg_end,
                                               const uint32_t* acc_flag,
                                               const uint32_t* id_local, int64_t n_commit,
                                               int32_t* vox_count, const int32_t* vox_slot,
                                               Slot* slots, uint32_t* seg_changed) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  int32_t vox = seg_vox[s];
  int32_t c = seg_newcount[s];
  const int32_t old = vox_count[vox];
  if (truncated) {
    c = old;
    for (uint32_t j = seg_start[s]; j < seg_end[s]; ++j) {
      uint32_t i = vals[j];
      if (acc_flag[i] && int64_t(id_local[i]) < n_commit) ++c;
    }
  }
  vox_count[vox] = c;
  slots[vox_slot[vox]].aux = c;
  seg_changed[s] = c != old ? 1u : 0u;
}

// ---------------------------------------------------------------- certificates
// Certificates an insert invalidates: those of the points within v of an
// added point, all of which lie in the 27 voxels around the added point's
// voxel.  Every voxel run that gained points marks itself and its existing
// neighbours with this insert's generation (plain stores of one value).
__global__ __launch_bounds__(kT) void k_cert_mark(int64_t n_seg, const int32_t* seg_vox,
                                                  const uint32_t* seg_changed,
                                                  const uint32_t* vox_nbr, uint32_t* mark,
                                                  uint32_t gen) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg || !seg_changed[s]) return;
  const int32_t V = seg_vox[s];
  mark[V] = gen;
  for (int d = 0; d < 26; ++d) {
    const uint32_t e = vox_nbr[int64_t(V) * 26 + d];
    if (e != kNbrNone) mark[e >> kNbrCountBits] = gen;
  }
}

// Certificate of every point of the marked voxels (all voxels when mark is
// null), one lane per voxel slot: the kCertK + 1 nearest other points
// within v by (d2, id) from the exact 27-voxel search (the point itself,
// and so kCertK + 2 entries, included), the first kCertK listed with their
// coordinates, rho half the distance of the next one (v/2 when there is
// none), shrunk by 2^-20 and rounded down to float so that it never exceeds
// the exact half distance.
__global__ __launch_bounds__(kT) void k_cert_build(MapView m, int64_t n_vox,
                                                   const uint32_t* mark, uint32_t gen,
                                                   CertRow* cert) {
  const int64_t pos = int64_t(blockIdx.x) * kT + threadIdx.x;
  const int64_t V = pos / m.nmax;
  if (V >= n_vox) return;
  if (mark && mark[V] != gen) return;
  if (pos - V * m.nmax >= m.vox_count[V]) return;
  const float4 p = m.vox_pts[pos];
  TopK<kCertK + 2> top;
  map_knn_query<kCertK + 2>(m, double(p.x), double(p.y), double(p.z), m.v * m.v, top);
  CertRow r;
  r.x = p.x;
  r.y = p.y;
  r.z = p.z;
  int n = 0;
  double next = -1.0;
#pragma unroll
  for (int t = 0; t < kCertK + 2; ++t) {
    if (top.pos[t] < 0 || top.pos[t] == int32_t(pos)) continue;
    if (n < kCertK) {
      const float4 u = m.vox_pts[top.pos[t]];
      r.nbr[n++] = make_float4(u.x, u.y, u.z, __int_as_float(top.pos[t]));
    } else if (next < 0.0) {
      next = top.d[t];
    }
  }
  for (int t = n; t < kCertK; ++t) r.nbr[t] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
  const double half = 0.5 * (next >= 0.0 ? sqrt(next) : m.v) * (1.0 - 0x1p-20);
  r.rho = __double2float_rd(half);
  cert[pos] = r;
}

// Neighbour table upkeep after an insert, one thread per touched voxel run:
// the voxel's entry (index and new count) is written into the row of every
// existing neighbour, and a new voxel's own row is filled from the hash.  An
// entry is written only by the thread of the voxel it names or of the voxel
// whose row it is, with the same (final) value, so the writes need no
// ordering.
__global__ __launch_bounds__(kT) void k_nbr_update(MapView m, int64_t n_seg, const int32_t* seg_vox,
                                                   const uint32_t* is_new, const uint64_t* vox_key,
                                                   const int32_t* vox_count, uint32_t* vox_nbr) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  const int32_t V = seg_vox[s];
  const bool fresh = is_new[s] != 0;
  const uint64_t key = vox_key[V];
  const int64_t kx = key_x(key), ky = key_y(key), kz = key_z(key);
  const uint32_t eV = (uint32_t(V) << kNbrCountBits) | uint32_t(vox_count[V]);
  for (int code = 0; code < 27; ++code) {
    if (code == 13) continue;
    int32_t cN;
    const int32_t N = map_find(m, kx + code / 9 - 1, ky + (code / 3) % 3 - 1, kz + code % 3 - 1, &cN);
    const int dir = nbr_dir(code), back = nbr_dir(26 - code);
    if (N >= 0) {
      vox_nbr[int64_t(N) * 26 + back] = eV;
      if (fresh) vox_nbr[int64_t(V) * 26 + dir] = (uint32_t(N) << kNbrCountBits) | uint32_t(cN);
    } else if (fresh) {
      vox_nbr[int64_t(V) * 26 + dir] = kNbrNone;
    }
  }
}

// ---------------------------------------------------------------- ghosts
// Ghost voxels are the empty voxels next to an occupied one.  Each has a
// neighbour-table row, so that a search from a point in an empty voxel reads
// its occupied neighbours from one row instead of probing the hash for each
// of the 26; a point whose voxel is neither occupied nor a ghost has no map
// point in its 27 voxels.  Ghosts are claimed around every new voxel, their
// rows filled from the hash, and the rows of the ghosts around every voxel
// whose count changed are updated with its new entry.  A ghost whose key
// later becomes occupied keeps its slot; the occupied voxel shadows it.

// Claims the empty neighbours of each new voxel run as ghosts (index from
// gcount; beyond ghost_cap a ghost gets no row and the host switches the
// ghosts off).
__global__ __launch_bounds__(kT) void k_ghost_claim(MapView m, int64_t n_seg,
                                                    const int32_t* seg_vox,
                                                    const uint32_t* is_new,
                                                    const uint64_t* vox_key, Slot* gslots,
                                                    uint64_t* gkey, uint32_t* gcount,
                                                    int64_t ghost_cap) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg || (is_new && !is_new[s])) return;
  const uint64_t key = vox_key[seg_vox[s]];
  const int64_t kx = key_x(key), ky = key_y(key), kz = key_z(key);
  for (int code = 0; code < 27; ++code) {
    if (code == 13) continue;
    const int64_t nx = kx + code / 9 - 1, ny = ky + (code / 3) % 3 - 1, nz = kz + code % 3 - 1;
    if (!key_ok(nx) || !key_ok(ny) || !key_ok(nz)) continue;
    int32_t c;
    if (map_find(m, nx, ny, nz, &c) >= 0) continue;
    const uint64_t nk = pack_key(nx, ny, nz);
    uint32_t h = voxel_hash(nx, ny, nz, m.glog2);
    for (uint32_t probe = 0; probe <= m.gmask; ++probe) {
      const unsigned long long old = atomicCAS(
          reinterpret_cast<unsigned long long*>(&gslots[h].key), (unsigned long long)kEmptyKey,
          (unsigned long long)nk);
      if (old == kEmptyKey) {
        const uint32_t g = atomicAdd(gcount, 1u);
        gslots[h].vox = int64_t(g) < ghost_cap ? int32_t(g) : -1;
        if (int64_t(g) < ghost_cap) gkey[g] = nk;
        break;
      }
      if (old == nk) break;
      h = (h + 1) & m.gmask;
    }
  }
}

// Full neighbour rows of the ghosts with index in [g0, min(*gcount, cap)).
__global__ __launch_bounds__(kT) void k_ghost_fill(MapView m, const uint64_t* gkey,
                                                   const uint32_t* gcount, int64_t g0,
                                                   int64_t n, int64_t ghost_cap,
                                                   uint32_t* gnbr) {
  const int64_t g = g0 + int64_t(blockIdx.x) * kT + threadIdx.x;
  const int64_t end = int64_t(*gcount) < ghost_cap ? int64_t(*gcount) : ghost_cap;
  if (g >= end || g >= g0 + n) return;
  const uint64_t key = gkey[g];
  const int64_t kx = key_x(key), ky = key_y(key), kz = key_z(key);
  for (int code = 0; code < 27; ++code) {
    if (code == 13) continue;
    int32_t c;
    const int32_t N = map_find(m, kx + code / 9 - 1, ky + (code / 3) % 3 - 1,
                               kz + code % 3 - 1, &c);
    gnbr[g * 26 + nbr_dir(code)] =
        N >= 0 ? (uint32_t(N) << kNbrCountBits) | uint32_t(c) : kNbrNone;
  }
}

// The entry of every voxel run whose count changed, written into the rows
// of the ghosts around it (one writer per entry, as in k_nbr_update).
__global__ __launch_bounds__(kT) void k_ghost_update(MapView m, int64_t n_seg,
                                                     const int32_t* seg_vox,
                                                     const uint32_t* seg_changed,
                                                     const uint64_t* vox_key,
                                                     const int32_t* vox_count, uint32_t* gnbr) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg || !seg_changed[s]) return;
  const int32_t V = seg_vox[s];
  const uint64_t key = vox_key[V];
  const int64_t kx = key_x(key), ky = key_y(key), kz = key_z(key);
  const uint32_t eV = (uint32_t(V) << kNbrCountBits) | uint32_t(vox_count[V]);
  for (int code = 0; code < 27; ++code) {
    if (code == 13) continue;
    const int32_t g = ghost_find(m, kx + code / 9 - 1, ky + (code / 3) % 3 - 1,
                                 kz + code % 3 - 1);
    if (g >= 0) gnbr[int64_t(g) * 26 + nbr_dir(26 - code)] = eV;
  }
}

// ---------------------------------------------------------------- ASMD
// Near-range points of the scan (sensor range <= r_near) and the distinct
// map-frame voxels they fall in, counted through a temporary hash set of
// keys (counters: [0] near points, [1] distinct voxels, [2] out of range).
__global__ __launch_bounds__(kT) void k_asmd_count(const float* xs, const float* xm, int64_t n,
                                                   double v, double rn2, uint64_t* set,
                                                   uint32_t set_mask, int set_log2,
                                                   uint32_t* counters) {
  const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  const double sx = xs[i], sy = xs[n + i], sz = xs[2 * n + i];
  const double mx = xm[i], my = xm[n + i], mz = xm[2 * n + i];
  if (!(isfinite(sx) && isfinite(sy) && isfinite(sz) && isfinite(mx) && isfinite(my) &&
        isfinite(mz)))
    return;
  if ((sx * sx + sy * sy) + sz * sz > rn2) return;
  int64_t kx, ky, kz;
  if (!voxel_index(mx, v, &kx) || !voxel_index(my, v, &ky) || !voxel_index(mz, v, &kz)) {
    atomicAdd(&counters[2], 1u);
    return;
  }
  atomicAdd(&counters[0], 1u);
  const uint64_t key = pack_key(kx, ky, kz);
  uint32_t h = voxel_hash(kx, ky, kz, set_log2);
  for (uint32_t probe = 0; probe <= set_mask; ++probe) {
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&set[h]),
                                             (unsigned long long)kEmptyKey,
                                             (unsigned long long)key);
    if (old == kEmptyKey) {
      atomicAdd(&counters[1], 1u);
      return;
    }
    if (old == key) return;
    h = (h + 1) & set_mask;
  }
}

// cap_i = clamp(floor(mean (1 - r_i / r_max) + 0.5), k, nmax), FP64 in this
// order (no contraction); non-finite points get k.  mean = near points /
// distinct near voxels from k_asmd_count's counters (nmax when none).
__global__ __launch_bounds__(kT) void k_asmd_caps(const float* xs, int64_t n,
                                                  const uint32_t* counters, double r_max,
                                                  int32_t k, int32_t nmax, int32_t* caps) {
  const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  const double mean =
      counters[1] > 0 ? double(counters[0]) / double(counters[1]) : double(nmax);
  const double sx = xs[i], sy = xs[n + i], sz = xs[2 * n + i];
  int32_t cap = k;
  if (isfinite(sx) && isfinite(sy) && isfinite(sz)) {
    const double r = sqrt((sx * sx + sy * sy) + sz * sz);
    const double c = floor(mean * (1.0 - r / r_max) + 0.5);
    cap = c < double(k) ? k : (c > double(nmax) ? nmax : int32_t(c));
  }
  caps[i] = cap;
}

// ---------------------------------------------------------------- eviction
// Keep flag of every map point: its voxel centre within radius of c.
__global__ __launch_bounds__(kT) void k_evict_keep(const float* pt_xyz, int64_t point_cap,
                                                   int64_t n, double v, double cx, double cy,
                                                   double cz, double r2, uint32_t* keep) {
  const int64_t id = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (id >= n) return;
  int64_t kx = 0, ky = 0, kz = 0;
  (void)voxel_index(double(pt_xyz[id]), v, &kx);
  (void)voxel_index(double(pt_xyz[point_cap + id]), v, &ky);
  (void)voxel_index(double(pt_xyz[2 * point_cap + id]), v, &kz);
  const double dx = (double(kx) + 0.5) * v - cx;
  const double dy = (double(ky) + 0.5) * v - cy;
  const double dz = (double(kz) + 0.5) * v - cz;
  keep[id] = ((dx * dx + dy * dy) + dz * dz <= r2) ? 1u : 0u;
}

// Survivors, in id order, into compact SoA coordinates and covariances.
__global__ __launch_bounds__(kT) void k_evict_gather(const float* pt_xyz, const float4* cov,
                                                     int64_t point_cap, int64_t n,
                                                     const uint32_t* keep, const uint32_t* nid,
                                                     int64_t n_keep, float* xyz_out,
                                                     float4* cov_out) {
  const int64_t id = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (id >= n || !keep[id]) return;
  const int64_t j = nid[id];
  xyz_out[j] = pt_xyz[id];
  xyz_out[n_keep + j] = pt_xyz[point_cap + id];
  xyz_out[2 * n_keep + j] = pt_xyz[2 * point_cap + id];
  cov_out[2 * j] = cov[2 * id];
  cov_out[2 * j + 1] = cov[2 * id + 1];
}

__global__ __launch_bounds__(kT) void k_evict_store(const float* xyz, int64_t n_keep,
                                                    int64_t point_cap, float* pt_xyz) {
  const int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n_keep) return;
  pt_xyz[j] = xyz[j];
  pt_xyz[point_cap + j] = xyz[n_keep + j];
  pt_xyz[2 * point_cap + j] = xyz[2 * n_keep + j];
}

// Every run of the rebuild is a new voxel, numbered in sorted key order.
__global__ __launch_bounds__(kT) void k_all_new(int64_t n_seg, uint32_t* is_new,
                                                uint32_t* rank) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  is_new[s] = 1u;
  rank[s] = uint32_t(s);
}

// Place the sorted survivors: a run's points keep their (id) order.
__global__ __launch_bounds__(kT) void k_bulk_place(const float* xyz, int64_t n,
                                                   const uint64_t* keys, const uint32_t* vals,
                                                   const uint32_t* head, const uint32_t* head_scan,
                                                   const uint32_t* seg_start,
                                                   const int32_t* seg_vox, int32_t nmax,
                                                   float4* vox_pts, int32_t* pt_loc) {
  const int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n || keys[j] == kEmptyKey) return;
  const uint32_t s = head_scan[j] + head[j] - 1;
  const int32_t pos = seg_vox[s] * nmax + int32_t(uint32_t(j) - seg_start[s]);
  const uint32_t id = vals[j];
  vox_pts[pos] = make_float4(xyz[id], xyz[n + id], xyz[2 * n + id], __int_as_float(int32_t(id)));
  pt_loc[id] = pos;
}

__global__ __launch_bounds__(kT) void k_bulk_counts(int64_t n_seg, const uint32_t* seg_start,
                                                    const uint32_t* seg_end,
                                                    const int32_t* seg_vox,
                                                    const int32_t* vox_slot, int32_t* vox_count,
                                                    Slot* slots) {
  const int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  const int32_t vox = seg_vox[s];
  const int32_t c = int32_t(seg_end[s] - seg_start[s]);
  vox_count[vox] = c;
  slots[vox_slot[vox]].aux = c;
}

// Covariances of map points [id0, id1): k nearest within v on the map.
template <int K>
__global__ __launch_bounds__(kT) void k_map_cov(MapView m, float4* cov, int64_t id0,
                                                int64_t id1, int32_t k, int32_t reg) {
  int64_t id = id0 + int64_t(blockIdx.x) * kT + threadIdx.x;
  if (id >= id1) return;
  double qx = m.pt_xyz[id], qy = m.pt_xyz[m.point_cap + id], qz = m.pt_xyz[2 * m.point_cap + id];
  TopK<K> top;
  map_knn_query<K>(m, qx, qy, qz, m.v * m.v, top);
  double c6[6] = {0, 0, 0, 0, 0, 0};
  bool ok = top.found() >= k;
  if (ok) regularised_cov<K>(top, k, [&](int32_t pos) { return m.vox_pts[pos]; }, c6, reg);
  cov[2 * id] = make_float4(float(c6[0]), float(c6[1]), float(c6[2]), float(c6[3]));
  cov[2 * id + 1] = make_float4(float(c6[4]), float(c6[5]), ok ? 1.0f : 0.0f, 0.0f);
}

// Copies of the covariance records of ids [id0, id1) at their vox_pts slots,
// so that a search reads a match's covariance beside its neighbours'.
__global__ __launch_bounds__(kT) void k_vox_cov(const float4* cov, const int32_t* pt_loc,
                                                int64_t id0, int64_t id1, float4* vox_cov) {
  const int64_t id = id0 + int64_t(blockIdx.x) * kT + threadIdx.x;
  if (id >= id1) return;
  const int64_t pos = pt_loc[id];
  vox_cov[2 * pos] = cov[2 * id];
  vox_cov[2 * pos + 1] = cov[2 * id + 1];
}

template <int K>
__global__ __launch_bounds__(kT) void k_map_knn(MapView m, const float* q, int64_t n, int32_t k,
                                                double r2, int32_t* idx, float* d2,
                                                int32_t* count) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  float x = q[i], y = q[n + i], z = q[2 * n + i];
  TopK<K> top;
  if (isfinite(x) && isfinite(y) && isfinite(z))
    map_knn_query<K>(m, double(x), double(y), double(z), r2, top);
  else
    top.init();
  int f = top.found();
  int c = f < k ? f : k;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    if (s < k) {
      idx[i * k + s] = s < c ? top.id[s] : -1;
      if (d2) d2[i * k + s] = s < c ? float(top.d[s]) : -1.0f;
    }
  }
  if (count) count[i] = c;
}

// ---------------------------------------------------------------- scan grid
// Each scan's own voxel grid is CSR: the points of all scans sorted by (scan,
// voxel key) (sorted[j] = x, y, z, original index bits), runs [seg_start,
// seg_end) of equal (scan, key), and a hash table from (scan, key) to run
// index (the scan id is kept in the slot's spare word and mixed into the hash).
struct GridView {
  const Slot* slots;
  const float4* sorted;
  const uint64_t* keys;       // sorted keys (kEmptyKey for non-finite points)
  const uint32_t* sid;        // scan id per sorted position (NULL: one scan)
  const uint32_t* seg_start;
  const uint32_t* seg_end;
  double v;          // neighbourhood radius (the voxel edge)
  double c;          // grid cell edge (v / 2 when v is a power of two, else v)
  double inv_c;
  int32_t pow2;
  const int64_t* part;        // scan offsets: the slots of each scan (NULL: one scan)
  uint32_t n_slots;           // two per point
  double mx;         // runs sorted by x up to a quantum: how far a later point of
                     // a run can lie below an earlier one along x (infinity:
                     // runs unordered)
  const uint32_t* head;       // 1 where a run starts
  const uint32_t* head_scan;  // exclusive prefix of head: run of j = head_scan + head - 1
  const uint2* nbt;           // per run, its 27 cells (code (ox+1)*9 + (oy+1)*3 + oz+1) as
                              // (start, count) in sorted; count 0: no run there
  const uint32_t* n_runs;     // the number of runs (device)
  float4* pk_B;               // the source packed for the align by sorted position
  float2* pk_C;               // (B, C as the align's pack writes them), or null
};

// The align's packed covariance words of sorted point j: B = (xx, or -1 when
// invalid, xy, xz, yy), C = (yz, zz), from the values written to cov6.
__device__ inline void write_packed(const GridView& g, int64_t j, const float c[6], bool ok) {
  if (!g.pk_B) return;
  g.pk_B[j] = make_float4(ok ? c[0] : -1.0f, c[1], c[2], c[3]);
  g.pk_C[j] = make_float2(c[4], c[5]);
}

// Slots of scan sc: two per point of the scan (its points are positions
// offsets[sc] .. offsets[sc + 1] of the sorted order, so at most half of its
// slots fill), or the whole table for a single scan.  Each scan's cells are
// hashed into its own stretch, so that the lookups of one scan, which the
// sorted order brings together, stay in a few MB of the table (one XCD's L2).
__device__ inline void grid_part(const GridView& g, uint32_t sc, uint32_t* base,
                                 uint32_t* size) {
  if (g.part) {
    const int64_t a = g.part[sc], b = g.part[sc + 1];
    *base = uint32_t(2 * a);
    *size = uint32_t(2 * (b - a));
  } else {
    *base = 0;
    *size = g.n_slots;
  }
}

__device__ inline uint32_t grid_hash(int64_t kx, int64_t ky, int64_t kz, uint32_t size) {
  const uint32_t h = (uint32_t(kx) * 73856093u) ^ (uint32_t(ky) * 19349669u) ^
                     (uint32_t(kz) * 83492791u);
  const uint32_t m = uint32_t((uint64_t(h) * 0x9E3779B97F4A7C15ull) >> 32);
  return uint32_t((uint64_t(m) * size) >> 32);
}

// Run of cell (kx, ky, kz) of scan sid: its start in sorted (or -1) and in
// *cnt its length.  A slot holds the cell's key, the run's start and its
// length (the scan is implied by the stretch of slots).
__device__ inline int32_t grid_find(const GridView& g, int64_t kx, int64_t ky, int64_t kz,
                                    uint32_t sid, int32_t* cnt) {
  *cnt = 0;
  if (!key_ok(kx) || !key_ok(ky) || !key_ok(kz)) return -1;
  const uint64_t key = pack_key(kx, ky, kz);
  uint32_t base, size;
  grid_part(g, sid, &base, &size);
  uint32_t s = grid_hash(kx, ky, kz, size);
  for (uint32_t probe = 0; probe < size; ++probe) {
    const Slot sl = load_slot(&g.slots[base + s]);
    if (sl.key == key) {
      *cnt = sl.aux;
      return sl.vox;
    }
    if (sl.key == kEmptyKey) return -1;
    s = s + 1 == size ? 0 : s + 1;
  }
  return -1;
}

// Scan id of each key-sorted point (binary search of its original index in
// the scan offsets); the result is the key of a second, stable sort.
__global__ __launch_bounds__(kT) void k_scan_ids(const uint32_t* vals, int64_t n,
                                                 const int64_t* offsets, int32_t S,
                                                 uint64_t* sid_key, uint32_t* pos) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  int64_t i = vals[j];
  int32_t lo = 0, hi = S;            // find s with offsets[s] <= i < offsets[s+1]
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (offsets[mid] <= i) lo = mid; else hi = mid;
  }
  sid_key[j] = uint64_t(lo);
  pos[j] = uint32_t(j);
}

__global__ __launch_bounds__(kT) void k_apply_perm(const uint32_t* perm, int64_t n,
                                                   const uint64_t* keys_in,
                                                   const uint32_t* vals_in, uint64_t* keys_out,
                                                   uint32_t* vals_out, const uint64_t* sid_key,
                                                   uint32_t* sid_out) {
  int64_t m = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (m >= n) return;
  uint32_t j = perm[m];
  keys_out[m] = keys_in[j];
  vals_out[m] = vals_in[j];
  sid_out[m] = uint32_t(sid_key[m]);
}

// ---------------------------------------------------------------- compact grid keys
// A batch's scan grid sorts its points by (scan, voxel key).  Keys limited to
// the batch's own range per axis need few bits (a sensor-frame scan of 120 m
// range at v = 1: 8 per axis), so one radix sort of (scan, kx - min, ky - min,
// kz - min) replaces a 63-bit sort followed by a sort by scan: the same
// order (both are lexicographic, stable on input order), in about half the
// passes.  The range comes from a two-level reduction (no same-address
// atomics); points without a finite, in-range key sort last in their scan.
constexpr int kRangePts = 16;                // points per lane of the range pass

// floor(x / v) as voxel_index computes it, through an exact multiply by 1/v
// when v is a power of two.
__device__ inline bool voxel_index_p2(double x, double v, double inv_v, bool pow2, int64_t* k) {
  const double f = floor(pow2 ? x * inv_v : x / v);
  if (!(f >= -double(kKeyBias) && f < double(kKeyBias))) return false;
  *k = int64_t(f);
  return true;
}

__global__ __launch_bounds__(kT) void k_key_range(const float* xyz, int64_t n, double v,
                                                  double inv_v, int32_t pow2, int32_t* part,
                                                  uint32_t* part_oor) {
  __shared__ int32_t s_r[kT / 64][6];
  __shared__ uint32_t s_o[kT / 64];
  int32_t r[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  uint32_t oor = 0;
  const int64_t base = int64_t(blockIdx.x) * (kT * kRangePts);
  for (int j = 0; j < kRangePts; ++j) {
    const int64_t i = base + j * kT + threadIdx.x;
    if (i >= n) break;
    const float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) continue;
    int64_t kx, ky, kz;
    if (voxel_index_p2(double(x), v, inv_v, pow2, &kx) &&
        voxel_index_p2(double(y), v, inv_v, pow2, &ky) &&
        voxel_index_p2(double(z), v, inv_v, pow2, &kz)) {
      r[0] = min(r[0], int32_t(kx)); r[3] = max(r[3], int32_t(kx));
      r[1] = min(r[1], int32_t(ky)); r[4] = max(r[4], int32_t(ky));
      r[2] = min(r[2], int32_t(kz)); r[5] = max(r[5], int32_t(kz));
    } else {
      ++oor;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    for (int a = 0; a < 3; ++a) {
      r[a] = min(r[a], __shfl_xor(r[a], d));
      r[3 + a] = max(r[3 + a], __shfl_xor(r[3 + a], d));
    }
    oor += uint32_t(__shfl_xor(int(oor), d));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int a = 0; a < 6; ++a) s_r[w][a] = r[a];
    s_o[w] = oor;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    int32_t x = s_r[0][threadIdx.x];
    for (int q = 1; q < kT / 64; ++q)
      x = threadIdx.x < 3 ? min(x, s_r[q][threadIdx.x]) : max(x, s_r[q][threadIdx.x]);
    part[int64_t(blockIdx.x) * 6 + threadIdx.x] = x;
  }
  if (threadIdx.x == 6) {
    uint32_t o = 0;
    for (int q = 0; q < kT / 64; ++q) o += s_o[q];
    part_oor[blockIdx.x] = o;
  }
}

// One block: the partial ranges in order into out[0..5], their sum of
// out-of-range counts into out[6].
__global__ __launch_bounds__(kT) void k_key_range_final(const int32_t* part,
                                                        const uint32_t* part_oor, int64_t nb,
                                                        int32_t* out) {
  __shared__ int32_t s_r[kT][6];
  __shared__ uint32_t s_o[kT];
  int32_t r[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  uint32_t oor = 0;
  for (int64_t b = threadIdx.x; b < nb; b += kT) {
    for (int a = 0; a < 3; ++a) {
      r[a] = min(r[a], part[b * 6 + a]);
      r[3 + a] = max(r[3 + a], part[b * 6 + 3 + a]);
    }
    oor += part_oor[b];
  }
  for (int a = 0; a < 6; ++a) s_r[threadIdx.x][a] = r[a];
  s_o[threadIdx.x] = oor;
  __syncthreads();
  if (threadIdx.x < 7) {
    if (threadIdx.x == 6) {
      uint32_t o = 0;
      for (int q = 0; q < kT; ++q) o += s_o[q];
      out[6] = int32_t(o);
    } else {
      int32_t x = s_r[0][threadIdx.x];
      for (int q = 1; q < kT; ++q)
        x = threadIdx.x < 3 ? min(x, s_r[q][threadIdx.x]) : max(x, s_r[q][threadIdx.x]);
      out[threadIdx.x] = x;
    }
  }
}

// Compact cell key: the cell's offsets from the batch's per-axis minima,
// bx, by, bz bits (each at least 2), laid out as 4 x 4 x 4 blocks of cells -
// the block's offsets (bx-2, by-2, bz-2 bits, x major) above the cell's place
// in the block (2 + 2 + 2 bits, x major) - so that sorted points fill whole
// blocks in turn: a stretch of the order is a compact patch of space.
struct CompactKey {
  int32_t mx, my, mz;   // per-axis minimum
  int32_t bx, by, bz;   // bits of x, y and z (>= 2)
  int32_t kb;           // key bits (x, y, z); 1 << kb marks an empty key
  int32_t fb;           // bits of the point's x within its cell, below the key
};

__device__ inline uint64_t compact_cell(const CompactKey& ck, int64_t cx, int64_t cy,
                                        int64_t cz) {
  const uint64_t hi = (uint64_t(cx >> 2) << (ck.by + ck.bz - 4)) |
                      (uint64_t(cy >> 2) << (ck.bz - 2)) | uint64_t(cz >> 2);
  return (hi << 6) | (uint64_t(cx & 3) << 4) | (uint64_t(cy & 3) << 2) | uint64_t(cz & 3);
}

__global__ __launch_bounds__(kT) void k_keys_compact(const float* xyz, int64_t n, double v,
                                                     double inv_v, int32_t pow2,
                                                     const int64_t* offsets, int32_t S,
                                                     CompactKey ck, uint64_t* keys,
                                                     uint32_t* vals) {
  const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  int32_t s = 0;
  if (offsets) {
    int32_t lo = 0, hi = S;            // offsets[s] <= i < offsets[s+1]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (offsets[mid] <= i) lo = mid; else hi = mid;
    }
    s = lo;
  }
  uint64_t key = uint64_t(1) << (ck.kb + ck.fb);
  const float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  int64_t kx, ky, kz;
  if (isfinite(x) && isfinite(y) && isfinite(z) &&
      voxel_index_p2(double(x), v, inv_v, pow2, &kx) &&
      voxel_index_p2(double(y), v, inv_v, pow2, &ky) &&
      voxel_index_p2(double(z), v, inv_v, pow2, &kz)) {
    // x / v less its floor is exact and non-decreasing in x within a cell,
    // so the fb bits below the key sort each run by x up to 2^-fb cells
    const double t = pow2 ? double(x) * inv_v : double(x) / v;
    const uint64_t xq = uint64_t(fmin((t - floor(t)) * ldexp(1.0, ck.fb), ldexp(1.0, ck.fb) - 1.0));
    key = (compact_cell(ck, kx - ck.mx, ky - ck.my, kz - ck.mz) << ck.fb) | xq;
  }
  keys[i] = (uint64_t(s) << (ck.kb + ck.fb + 1)) | key;
  vals[i] = uint32_t(i);
}

// Sorted compact keys back to full keys (kEmptyKey for the empty ones) and
// scan ids.
__global__ __launch_bounds__(kT) void k_keys_expand(const uint64_t* ckeys, int64_t n,
                                                    CompactKey ck, uint64_t* keys,
                                                    uint32_t* sid) {
  const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= n) return;
  const uint64_t c = ckeys[i] >> ck.fb;
  const uint64_t k = c & ((uint64_t(2) << ck.kb) - 1);
  if (sid) sid[i] = uint32_t(c >> (ck.kb + 1));
  if (k >> ck.kb) {
    keys[i] = kEmptyKey;
  } else {
    const uint64_t hi = k >> 6;
    const int64_t hx = int64_t(hi >> (ck.by + ck.bz - 4));
    const int64_t hy = int64_t((hi >> (ck.bz - 2)) & ((uint64_t(1) << (ck.by - 2)) - 1));
    const int64_t hz = int64_t(hi & ((uint64_t(1) << (ck.bz - 2)) - 1));
    const int64_t kx = ((hx << 2) | int64_t((k >> 4) & 3)) + ck.mx;
    const int64_t ky = ((hy << 2) | int64_t((k >> 2) & 3)) + ck.my;
    const int64_t kz = ((hz << 2) | int64_t(k & 3)) + ck.mz;
    keys[i] = pack_key(kx, ky, kz);
  }
}

__global__ __launch_bounds__(kT) void k_grid_heads(const uint64_t* keys, const uint32_t* sid,
                                                   int64_t n, uint32_t* head) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  uint64_t k = keys[j];
  bool h = k != kEmptyKey &&
           (j == 0 || keys[j - 1] != k || (sid && sid[j - 1] != sid[j]));
  head[j] = h ? 1u : 0u;
}

__global__ __launch_bounds__(kT) void k_grid_bounds(const uint64_t* keys, const uint32_t* sid,
                                                    int64_t n, const uint32_t* head,
                                                    const uint32_t* head_scan,
                                                    uint32_t* seg_start, uint32_t* seg_end) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  uint64_t k = keys[j];
  if (k == kEmptyKey) return;
  uint32_t s = head_scan[j] + head[j] - 1;
  if (head[j]) seg_start[s] = uint32_t(j);
  if (j == n - 1 || keys[j + 1] != k || (sid && sid[j + 1] != sid[j]))
    seg_end[s] = uint32_t(j + 1);
}

// Sorted points as float4 (and, when order is not null, the sorted order
// itself: order[j] = the original index of sorted point j), blocks dealt to
// the XCDs in contiguous ranges (a scan's points stay in the scan's index
// range, so each XCD gathers from the few MB of its own scans).
__global__ __launch_bounds__(kT) void k_gather_sorted(const float* xyz, int64_t n,
                                                      const uint32_t* vals, float4* sorted,
                                                      uint32_t* order) {
  const int64_t nb = (n + kT - 1) / kT, chunk = (nb + 7) >> 3;
  const int64_t j = (int64_t(blockIdx.x & 7) * chunk + (blockIdx.x >> 3)) * kT + threadIdx.x;
  if ((blockIdx.x >> 3) >= chunk || j >= n) return;
  uint32_t i = vals[j];
  sorted[j] = make_float4(xyz[i], xyz[n + i], xyz[2 * n + i], __int_as_float(int32_t(i)));
  if (order) order[j] = i;
}

// The run count stays on the device: the grid-wide kernels over runs are
// persistent grids (kGridBlocks blocks, a multiple of 8) that split the items
// into eight contiguous ranges, one per XCD, and walk their range in steps
// of the XCD's blocks.
constexpr int kGridBlocks = 8 * 1024;

template <class F>
__device__ inline void xcd_ranges(int64_t total, F f) {
  const int64_t chunk = (total + 7) >> 3;
  const int64_t lo = int64_t(blockIdx.x & 7) * chunk, hi = min(lo + chunk, total);
  const int64_t step = int64_t(gridDim.x >> 3) * kT;
  for (int64_t t = lo + int64_t(blockIdx.x >> 3) * kT + threadIdx.x; t < hi; t += step) f(t);
}

// Run r into the slots of its scan (one XCD fills one scan's slots at a time).
__device__ inline void grid_claim_run(const GridView& g, Slot* slots, int64_t r) {
  const uint32_t j = g.seg_start[r];
  const uint64_t key = g.keys[j];
  const uint32_t sc = g.sid ? g.sid[j] : 0u;
  uint32_t base, size;
  grid_part(g, sc, &base, &size);
  uint32_t h = grid_hash(key_x(key), key_y(key), key_z(key), size);
  const uint32_t cnt = g.seg_end[r] - j;   // >= 1, so never the empty word
  // every run is a different cell, so a slot is claimed on its length word
  // alone (a 32-bit compare-and-swap); key and start follow as plain stores,
  // read only by later kernels
  for (uint32_t probe = 0; probe < size; ++probe) {
    const uint32_t old = atomicCAS(reinterpret_cast<uint32_t*>(&slots[base + h].aux),
                                   0xFFFFFFFFu, cnt);
    if (old == 0xFFFFFFFFu) {
      slots[base + h].key = key;
      slots[base + h].vox = int32_t(j);
      return;
    }
    h = h + 1 == size ? 0 : h + 1;
  }
}

__global__ __launch_bounds__(kT) void k_grid_claim(GridView g, Slot* slots) {
  xcd_ranges(*g.n_runs, [&](int64_t r) { grid_claim_run(g, slots, r); });
}

// Neighbour table of the runs: per run, the (start, count) of the run of the
// same scan in each of its 27 cells, so that a point's search reads its
// cells from its run's row instead of probing the hash for each.  One thread
// per (run, cell) entry t, the entries in XCD ranges (one XCD probes one
// scan's stretch of slots at a time); the rows are written with non-temporal
// stores so that they stream past the L2 holding the slots.
__device__ inline void grid_nbr_entry(const GridView& g, uint2* nbt, int64_t t) {
  const int64_t r = t / 27;
  const int code = int(t - r * 27);
  const uint32_t s0 = g.seg_start[r];
  uint32_t a = s0, c = g.seg_end[r] - s0;
  if (code != 13) {
    const uint64_t key = g.keys[s0];
    const uint32_t sc = g.sid ? g.sid[s0] : 0u;
    int32_t cnt;
    const int32_t f = grid_find(g, key_x(key) + code / 9 - 1, key_y(key) + (code / 3) % 3 - 1,
                                key_z(key) + code % 3 - 1, sc, &cnt);
    a = f < 0 ? 0u : uint32_t(f);
    c = f < 0 ? 0u : uint32_t(cnt);
  }
  __builtin_nontemporal_store(a, &nbt[t].x);
  __builtin_nontemporal_store(c, &nbt[t].y);
}

__global__ __launch_bounds__(kT) void k_grid_nbr_table(GridView g, uint2* nbt) {
  xcd_ranges(int64_t(*g.n_runs) * 27, [&](int64_t t) { grid_nbr_entry(g, nbt, t); });
}

// Squared face distance as a float never above the FP64 value (rounded
// down, shrunk by 2^-20 to cover the float sums of three terms).
__device__ inline float face_lb(double g) { return __double2float_rd(g * g) * (1.0f - 0x1p-20f); }

// Covariances, one wave per grid run (the points of one scan in one voxel of
// edge v).  All of a run's queries share one 27-voxel neighbourhood (every
// point within v of them lies in it), so the wave reads the run's row of the
// neighbour table once and walks each needed voxel's points at wave-uniform
// addresses, every lane testing the same candidate against its own query; a
// voxel that no lane's current k-th distance can reach is skipped.  Exact,
// like the per-point search: ranking by (d2, id) over a superset of the
// candidates.  Only runs of at least `dense` points are taken: in sparse runs
// most lanes would idle while the wave walks the neighbourhood.
template <int K>
__device__ inline void grid_cov_run(const GridView& g, int64_t sg, int32_t dense, int64_t n,
                                    int32_t k, int32_t reg, float* cov6, uint8_t* valid,
                                    int32_t* nb_start, int32_t* nb_cnt) {
  const int lane = threadIdx.x;
  __syncthreads();   // the previous run's readers of nb_start and nb_cnt are done
  const uint32_t s0 = g.seg_start[sg], s1 = g.seg_end[sg];
  if (int64_t(s1 - s0) < dense) return;   // sparse runs: the per-point search
  const uint64_t key = g.keys[s0];
  const int64_t kx = key_x(key), ky = key_y(key), kz = key_z(key);
  if (lane < 27) {   // the run's row of the neighbour table
    const uint2 e = g.nbt[sg * 27 + lane];
    nb_start[lane] = e.y ? int32_t(e.x) : -1;
    nb_cnt[lane] = int32_t(e.y);
  }
  __syncthreads();
  const double v = g.v, r2 = v * v, slack = 1e-7 * v;
  const double bx = double(kx) * v, by = double(ky) * v, bz = double(kz) * v;
  for (uint32_t q0 = s0; q0 < s1; q0 += 64) {
    const uint32_t j = q0 + uint32_t(lane);
    const bool act = j < s1;
    const float4 me = g.sorted[act ? j : s0];
    const double qx = me.x, qy = me.y, qz = me.z;
    float gl2[3], gh2[3];
    gl2[0] = face_lb(fmax(qx - bx - slack, 0.0)); gh2[0] = face_lb(fmax(bx + v - qx - slack, 0.0));
    gl2[1] = face_lb(fmax(qy - by - slack, 0.0)); gh2[1] = face_lb(fmax(by + v - qy - slack, 0.0));
    gl2[2] = face_lb(fmax(qz - bz - slack, 0.0)); gh2[2] = face_lb(fmax(bz + v - qz - slack, 0.0));
    Query q = make_query(qx, qy, qz, r2);
    TopK<K> top;
    top.init();
    for (int rank = 0; rank < 27; ++rank) {
      const int code = rank == 0 ? 13 : nbr_code(rank);
      const int32_t cnt = __builtin_amdgcn_readfirstlane(nb_cnt[code]);
      if (cnt == 0) continue;
      bool need = act;
      if (rank > 0) {
        const int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
        const float lb = (ox < 0 ? gl2[0] : (ox > 0 ? gh2[0] : 0.0f)) +
                         (oy < 0 ? gl2[1] : (oy > 0 ? gh2[1] : 0.0f)) +
                         (oz < 0 ? gl2[2] : (oz > 0 ? gh2[2] : 0.0f));
        need = need && double(lb) <= fmin(r2, top.bound());
      }
      if (!__any(need)) continue;
      const int32_t st = __builtin_amdgcn_readfirstlane(nb_start[code]);
      scan_voxel_points<K>(g.sorted, st, cnt, q, r2, top);
    }
    if (act) {
      double c6[6] = {0, 0, 0, 0, 0, 0};
      const bool ok = top.found() >= k;
      if (ok) regularised_cov<K>(top, k, [&](int32_t pos) { return g.sorted[pos]; }, c6, reg);
      const int64_t i = __float_as_int(me.w);
      float cf[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        cf[t] = float(c6[t]);
        cov6[t * n + i] = cf[t];
      }
      valid[i] = ok ? 1 : 0;
      write_packed(g, j, cf, ok);
    }
  }
}

template <int K>
__global__ __launch_bounds__(64) void k_grid_cov_wave(GridView g, int32_t dense, int64_t n,
                                                      int32_t k, int32_t reg, float* cov6,
                                                      uint8_t* valid) {
  __shared__ int32_t nb_start[27];
  __shared__ int32_t nb_cnt[27];
  // the runs in eight contiguous ranges, one per XCD; each block of an XCD
  // takes every (gridDim / 8)-th run of its range
  const int64_t n_seg = *g.n_runs;
  const int64_t chunk = (n_seg + 7) >> 3;
  const int64_t lo = int64_t(blockIdx.x & 7) * chunk, hi = min(lo + chunk, n_seg);
  for (int64_t sg = lo + (blockIdx.x >> 3); sg < hi; sg += gridDim.x >> 3)
    grid_cov_run<K>(g, sg, dense, n, k, reg, cov6, valid, nb_start, nb_cnt);
}

// Covariance of every scan point from its k nearest points of the same scan
// within v, one point per lane over the 27 voxels (processed in sorted order
// for locality; written at the original index).  Points of runs with at
// least `dense` points (dense > 0) are left to k_grid_cov_wave.  Non-finite
// points get the zero covariance and the invalid flag.
// Waves per SIMD asked of the per-point covariance search (latency-bound
// gathers, as in the linearisation).
constexpr int kCovMinWaves = 5;

template <int K>
__global__ __launch_bounds__(kT, kCovMinWaves) void k_grid_cov(GridView g, int32_t dense, int64_t n,
                                                               int32_t k, int32_t reg,
                                                               float* cov6, uint8_t* valid) {
  // blocks dealt to the eight XCDs in contiguous ranges of the sorted
  // points: the neighbour voxels a block reads are those of the blocks
  // around it, which then share that XCD's L2
  const int64_t nb = (n + kT - 1) / kT, chunk = (nb + 7) >> 3;
  const int64_t b = int64_t(blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  const int64_t j = b * kT + threadIdx.x;
  if ((blockIdx.x >> 3) >= chunk || j >= n) return;
  const float4 me = g.sorted[j];
  if (g.keys[j] == kEmptyKey) {   // a non-finite point: zero covariance, invalid
    const int64_t i = __float_as_int(me.w);
#pragma unroll
    for (int t = 0; t < 6; ++t) cov6[t * n + i] = 0.0f;
    valid[i] = 0;
    const float z[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    write_packed(g, j, z, false);
    return;
  }
  const double qx = me.x, qy = me.y, qz = me.z;
  // the cells around the point's own cell (the cell of its run's key: the
  // same coordinates and cell edge) from its run's row of the neighbour table
  const uint2* row = g.nbt + int64_t(g.head_scan[j] + g.head[j] - 1) * 27;
  if (dense > 0 && int32_t(row[13].y) >= dense) return;
  TopK<K> top;
  knn_cells27<K>(qx, qy, qz, g.c, g.inv_c, g.pow2 != 0, g.v * g.v, g.sorted, int32_t(j), g.mx,
                 [&](int code, int32_t* cnt) {
                   const uint2 e = row[code];
                   *cnt = int32_t(e.y);
                   return e.y ? int32_t(e.x) : int32_t(-1);
                 },
                 top);
  double c6[6] = {0, 0, 0, 0, 0, 0};
  const bool ok = top.found() >= k;
  if (ok) regularised_cov<K>(top, k, [&](int32_t pos) { return g.sorted[pos]; }, c6, reg);
  const int64_t i = __float_as_int(me.w);
  const float f0 = float(c6[0]), f1 = float(c6[1]), f2 = float(c6[2]), f3 = float(c6[3]),
              f4 = float(c6[4]), f5 = float(c6[5]);
  if (g.pk_B) {   // the align's packed words at the sorted position (n < 2^31)
    const uint32_t j32 = uint32_t(j);
    g.pk_B[j32] = make_float4(ok ? f0 : -1.0f, f1, f2, f3);
    g.pk_C[j32] = make_float2(f4, f5);
  }
  cov6[i] = f0;
  cov6[n + i] = f1;
  cov6[2 * n + i] = f2;
  cov6[3 * n + i] = f3;
  cov6[4 * n + i] = f4;
  cov6[5 * n + i] = f5;
  valid[i] = ok ? 1 : 0;
}

__global__ __launch_bounds__(kT) void k_probe_stats(const Slot* slots, int64_t n_slots,
                                                    uint32_t slot_mask, int log2_slots,
                                                    unsigned long long* sum,
                                                    uint32_t* maxp) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_slots) return;
  uint64_t key = slots[s].key;
  if (key == kEmptyKey) return;
  uint32_t h = voxel_hash(key_x(key), key_y(key), key_z(key), log2_slots);
  uint32_t len = ((uint32_t(s) - h) & slot_mask) + 1;
  atomicAdd(sum, (unsigned long long)len);
  atomicMax(maxp, len);
}

__global__ __launch_bounds__(kT) void k_export(const float4* cov, const float* pt_xyz,
                                               int64_t point_cap, int64_t N, float* xyz,
                                               float* cov6, uint8_t* valid) {
  int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= N) return;
  if (xyz) {
    xyz[i] = pt_xyz[i];
    xyz[N + i] = pt_xyz[point_cap + i];
    xyz[2 * N + i] = pt_xyz[2 * point_cap + i];
  }
  float4 a = cov[2 * i], b = cov[2 * i + 1];
  if (cov6) {
    cov6[i] = a.x;
    cov6[N + i] = a.y;
    cov6[2 * N + i] = a.z;
    cov6[3 * N + i] = a.w;
    cov6[4 * N + i] = b.x;
    cov6[5 * N + i] = b.y;
  }
  if (valid) valid[i] = b.z != 0.0f ? 1 : 0;
}

// ---------------------------------------------------------------- fine index
// Fine cell key of every map point (cells of v/2, exact: v is a power of
// two); a key outside the 21-bit range is counted and disables the index.
__global__ __launch_bounds__(kT) void k_fine_keys(const float* pt_xyz, int64_t point_cap,
                                                  int64_t n, double inv_fc, uint64_t* keys,
                                                  uint32_t* vals, uint32_t* counters) {
  int64_t id = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (id >= n) return;
  const double x = pt_xyz[id], y = pt_xyz[point_cap + id], z = pt_xyz[2 * point_cap + id];
  const double fx = floor(x * inv_fc), fy = floor(y * inv_fc), fz = floor(z * inv_fc);
  const double lim = double(kKeyBias);
  uint64_t key = kEmptyKey;
  if (fx >= -lim && fx < lim && fy >= -lim && fy < lim && fz >= -lim && fz < lim)
    key = pack_key(int64_t(fx), int64_t(fy), int64_t(fz));
  else
    atomicAdd(&counters[1], 1u);
  keys[id] = key;
  vals[id] = uint32_t(id);
}

__global__ __launch_bounds__(kT) void k_fine_fill(const float* pt_xyz, int64_t point_cap,
                                                  int64_t n, const uint32_t* vals,
                                                  float4* fine_pts) {
  int64_t j = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (j >= n) return;
  const uint32_t id = vals[j];
  fine_pts[j] = make_float4(pt_xyz[id], pt_xyz[point_cap + id], pt_xyz[2 * point_cap + id],
                            __int_as_float(int32_t(id)));
}

__global__ __launch_bounds__(kT) void k_fine_claim(Slot* slots, uint32_t slot_mask,
                                                   int log2_slots, const uint64_t* keys,
                                                   const uint32_t* seg_start,
                                                   const uint32_t* seg_end, int64_t n_seg) {
  int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (s >= n_seg) return;
  const uint64_t key = keys[seg_start[s]];
  uint32_t h = voxel_hash(key_x(key), key_y(key), key_z(key), log2_slots);
  for (uint32_t probe = 0; probe <= slot_mask; ++probe) {
    unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&slots[h].key),
                                       (unsigned long long)kEmptyKey,
                                       (unsigned long long)key);
    if (old == kEmptyKey) {
      slots[h].vox = int32_t(seg_start[s]);
      slots[h].aux = int32_t(seg_end[s] - seg_start[s]);
      return;
    }
    h = (h + 1) & slot_mask;
  }
}

template <class F>
far_status_t dispatch_k(int32_t k, F&& f) {
  if (k <= 1) return f(std::integral_constant<int, 1>());
  if (k <= 4) return f(std::integral_constant<int, 4>());
  if (k == 5) return f(std::integral_constant<int, 5>());
  if (k <= 8) return f(std::integral_constant<int, 8>());
  if (k <= 10) return f(std::integral_constant<int, 10>());
  if (k <= 16) return f(std::integral_constant<int, 16>());
  return f(std::integral_constant<int, 32>());
}

// Keys, stable sort and runs of a point batch: the common front half of the
// insert and of the scan covariances.
struct Runs {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* head;
  uint32_t* head_scan;
  uint32_t* seg_start;
  uint32_t* seg_end;
  uint32_t* counters;   // [0] non-finite, [1] out of range, [2] runs
};

far_status_t build_runs(const float* xyz, int64_t n, double v, hipStream_t st, Scratch& scr,
                        Runs& r) {
  uint64_t* keys_alt;
  uint32_t* vals_alt;
  FAR_TRY(scr.get(&r.keys, size_t(n)));
  FAR_TRY(scr.get(&r.vals, size_t(n)));
  FAR_TRY(scr.get(&keys_alt, size_t(n)));
  FAR_TRY(scr.get(&vals_alt, size_t(n)));
  FAR_TRY(scr.get(&r.head, size_t(n)));
  FAR_TRY(scr.get(&r.head_scan, size_t(n)));
  FAR_TRY(scr.get(&r.seg_start, size_t(n)));
  FAR_TRY(scr.get(&r.seg_end, size_t(n)));
  FAR_TRY(scr.get(&r.counters, 4));
  FAR_HIP(hipMemsetAsync(r.counters, 0, 4 * sizeof(uint32_t), st));
  k_keys<<<blocks_for(n), kT, 0, st>>>(xyz, n, v, r.keys, r.vals, r.counters);
  FAR_HIP(hipGetLastError());
  FAR_TRY(radix_sort_pairs(r.keys, r.vals, keys_alt, vals_alt, n, kKeyBits, st, scr));
  k_heads<<<blocks_for(n), kT, 0, st>>>(r.keys, n, r.head);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(r.head, r.head_scan, n, r.counters + 2, st, scr));
  k_seg_bounds<<<blocks_for(n), kT, 0, st>>>(r.keys, n, r.head, r.head_scan, r.seg_start,
                                              r.seg_end);
  FAR_HIP(hipGetLastError());
  return FAR_OK;
}

inline int ceil_log2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

}  // namespace

// Covariance regularisation of every covariance computed from now on
// (far_set_covariance_regularisation): FAR_REG_EQ1 or FAR_REG_PLANE.
int32_t g_cov_reg = FAR_REG_EQ1;

far_status_t map_covariances(const MapView& m, float4* cov_out, int64_t id0, int64_t id1,
                             int32_t k, hipStream_t st) {
  if (id1 <= id0) return FAR_OK;
  return dispatch_k(k, [&](auto KK) -> far_status_t {
    constexpr int K = decltype(KK)::value;
    k_map_cov<K><<<blocks_for(id1 - id0), kT, 0, st>>>(m, cov_out, id0, id1, k, g_cov_reg);
    FAR_HIP(hipGetLastError());
    return FAR_OK;
  });
}

far_status_t fine_build(far_map_s* m, hipStream_t st) {
  if (m->fine_ok || m->n_points == 0) return FAR_OK;
  int e2 = 0;
  if (std::frexp(m->p.voxel_size, &e2) != 0.5) return FAR_OK;   // not a power of two
  const int64_t n = m->n_points;
  Scratch scr(st);
  uint64_t *keys, *keys_alt;
  uint32_t *vals, *vals_alt, *head, *head_scan, *seg_start, *seg_end, *counters;
  FAR_TRY(scr.get(&keys, size_t(n)));
  FAR_TRY(scr.get(&keys_alt, size_t(n)));
  FAR_TRY(scr.get(&vals, size_t(n)));
  FAR_TRY(scr.get(&vals_alt, size_t(n)));
  FAR_TRY(scr.get(&head, size_t(n)));
  FAR_TRY(scr.get(&head_scan, size_t(n)));
  FAR_TRY(scr.get(&seg_start, size_t(n)));
  FAR_TRY(scr.get(&seg_end, size_t(n)));
  FAR_TRY(scr.get(&counters, 4));
  FAR_HIP(hipMemsetAsync(counters, 0, 4 * sizeof(uint32_t), st));
  const double inv_fc = 2.0 / m->p.voxel_size;
  k_fine_keys<<<blocks_for(n), kT, 0, st>>>(m->pt_xyz, m->p.point_capacity, n, inv_fc, keys,
                                            vals, counters);
  FAR_HIP(hipGetLastError());
  FAR_TRY(radix_sort_pairs(keys, vals, keys_alt, vals_alt, n, kKeyBits, st, scr));
  k_heads<<<blocks_for(n), kT, 0, st>>>(keys, n, head);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(head, head_scan, n, counters + 2, st, scr));
  k_seg_bounds<<<blocks_for(n), kT, 0, st>>>(keys, n, head, head_scan, seg_start, seg_end);
  FAR_HIP(hipGetLastError());
  uint32_t h_cnt[4];
  FAR_HIP(hipMemcpyAsync(h_cnt, counters, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  if (h_cnt[1] > 0) return FAR_OK;                    // out of the fine key range
  const int64_t n_seg = h_cnt[2];
  FAR_HIP(hipMemsetAsync(m->fine_slots, 0xFF, size_t(m->fine_nslots) * sizeof(Slot), st));
  k_fine_claim<<<blocks_for(n_seg), kT, 0, st>>>(m->fine_slots, uint32_t(m->fine_nslots - 1),
                                                 m->fine_log2, keys, seg_start, seg_end, n_seg);
  FAR_HIP(hipGetLastError());
  k_fine_fill<<<blocks_for(n), kT, 0, st>>>(m->pt_xyz, m->p.point_capacity, n, vals,
                                            m->fine_pts);
  FAR_HIP(hipGetLastError());
  m->fine_ok = true;
  return FAR_OK;
}

// No ghosts (the voxel structures were cleared): an empty table, ghosts on.
far_status_t ghosts_reset(far_map_s* m, hipStream_t st) {
  FAR_HIP(hipMemsetAsync(m->gslots, 0xFF, size_t(m->gslots_n) * sizeof(Slot), st));
  FAR_HIP(hipMemsetAsync(m->gcount, 0, sizeof(uint32_t), st));
  m->n_ghosts = 0;
  m->ghost_ok = true;
  return FAR_OK;
}

// Ghost upkeep after the voxels of runs seg_vox changed: claim the empty
// neighbours of the new voxels (every run when is_new is NULL), fill the new
// ghosts' rows, and update the rows around the changed voxels (when
// seg_changed is given); then (one small copy; the callers synchronise
// anyway) the host learns the ghost count and switches the ghosts off when
// they no longer fit.
far_status_t ghosts_update(far_map_s* m, int64_t n_seg, const int32_t* seg_vox,
                           const uint32_t* is_new, const uint32_t* seg_changed, int64_t n_new,
                           hipStream_t st) {
  if (!m->ghost_ok || n_seg == 0) return FAR_OK;
  const MapView mv = m->view();
  k_ghost_claim<<<blocks_for(n_seg), kT, 0, st>>>(mv, n_seg, seg_vox, is_new, m->vox_key,
                                                  m->gslots, m->gkey, m->gcount, m->ghost_cap);
  FAR_HIP(hipGetLastError());
  const int64_t fresh = 26 * n_new;   // at most this many new ghosts
  if (fresh > 0) {
    k_ghost_fill<<<blocks_for(fresh), kT, 0, st>>>(mv, m->gkey, m->gcount, m->n_ghosts, fresh,
                                                   m->ghost_cap, m->gnbr);
    FAR_HIP(hipGetLastError());
  }
  if (seg_changed) {
    k_ghost_update<<<blocks_for(n_seg), kT, 0, st>>>(mv, n_seg, seg_vox, seg_changed,
                                                     m->vox_key, m->vox_count, m->gnbr);
    FAR_HIP(hipGetLastError());
  }
  uint32_t h = 0;
  FAR_HIP(hipMemcpyAsync(&h, m->gcount, sizeof(h), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  m->n_ghosts = h;
  if (int64_t(h) > m->ghost_cap) m->ghost_ok = false;
  return FAR_OK;
}

}  // namespace far

using namespace far;

extern "C" {

const char* far_status_str(far_status_t s) {
  switch (s) {
    case FAR_OK: return "ok";
    case FAR_E_INVALID: return "invalid argument";
    case FAR_E_CAPACITY: return "capacity exceeded";
    case FAR_E_HIP: return "HIP runtime error";
    case FAR_E_NOT_PD: return "H not positive definite";
    case FAR_E_FEW_CORR: return "too few correspondences";
    case FAR_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* far_last_error(void) { return g_err; }

far_status_t far_map_create(const far_map_params_t* params, far_stream_t stream,
                            far_map_t* out) {
  if (!params || !out) {
    set_error("far_map_create: null argument");
    return FAR_E_INVALID;
  }
  *out = nullptr;
  far_map_params_t p = *params;
  if (!(p.voxel_size > 0.0) || !std::isfinite(p.voxel_size) || p.max_pts_per_voxel < 1 ||
      p.max_pts_per_voxel > 64 || p.point_capacity < 1 || p.point_capacity >= (int64_t(1) << 31) ||
      p.k_cov < 1 || p.k_cov > 32 || !std::isfinite(p.min_spacing)) {
    set_error("far_map_create: parameter out of range");
    return FAR_E_INVALID;
  }
  // the neighbour table packs a voxel index into 25 bits
  if (p.voxel_capacity <= 0)
    p.voxel_capacity = std::min<int64_t>(p.point_capacity, (int64_t(1) << 25) - 1);
  if (p.voxel_capacity >= (int64_t(1) << 25) ||
      p.voxel_capacity * p.max_pts_per_voxel >= (int64_t(1) << 31)) {
    set_error("far_map_create: need voxel_capacity < 2^25 and voxel_capacity * "
              "max_pts_per_voxel < 2^31");
    return FAR_E_INVALID;
  }
  hipStream_t st = S(stream);
  far_map_s* m = new far_map_s();
  m->p = p;
  m->dmin = p.min_spacing < 0 ? p.voxel_size / std::sqrt(double(p.max_pts_per_voxel))
                              : p.min_spacing;
  m->voxel_cap = p.voxel_capacity;
  m->log2_slots = ceil_log2(2 * p.voxel_capacity);
  if (m->log2_slots < 10) m->log2_slots = 10;
  m->slots = int64_t(1) << m->log2_slots;
  if (hipGetDevice(&m->device) != hipSuccess) m->device = 0;
  auto fail = [&](hipError_t e, const char* what) {
    far_map_destroy(m);
    return hip_fail(e, what, __FILE__, __LINE__);
  };
  hipError_t e;
  size_t b_slots = size_t(m->slots) * sizeof(Slot);
  size_t b_cnt = size_t(m->voxel_cap) * sizeof(int32_t);
  size_t b_key = size_t(m->voxel_cap) * sizeof(uint64_t);
  size_t b_pts = size_t(m->voxel_cap) * p.max_pts_per_voxel * sizeof(float4);
  size_t b_cov = size_t(p.point_capacity) * 2 * sizeof(float4);
  size_t b_vcov = size_t(m->voxel_cap) * p.max_pts_per_voxel * 2 * sizeof(float4);
  size_t b_nbr = size_t(m->voxel_cap) * 26 * sizeof(uint32_t);
  size_t b_xyz = size_t(p.point_capacity) * 3 * sizeof(float);
  size_t b_loc = size_t(p.point_capacity) * sizeof(int32_t);
  size_t b_vslot = size_t(m->voxel_cap) * sizeof(int32_t);
  size_t b_cert = size_t(m->voxel_cap) * p.max_pts_per_voxel * sizeof(CertRow);
  size_t b_mark = size_t(m->voxel_cap) * sizeof(uint32_t);
  // ghosts: four per voxel of capacity (a surface map has about two)
  m->ghost_cap = 4 * m->voxel_cap;
  m->glog2 = ceil_log2(2 * m->ghost_cap);
  if (m->glog2 < 10) m->glog2 = 10;
  m->gslots_n = int64_t(1) << m->glog2;
  size_t b_gslots = size_t(m->gslots_n) * sizeof(Slot);
  size_t b_gkey = size_t(m->ghost_cap) * sizeof(uint64_t);
  size_t b_gnbr = size_t(m->ghost_cap) * 26 * sizeof(uint32_t);
  m->fine_log2 = ceil_log2(2 * p.point_capacity);
  if (m->fine_log2 < 10) m->fine_log2 = 10;
  m->fine_nslots = int64_t(1) << m->fine_log2;
  size_t b_fpts = size_t(p.point_capacity) * sizeof(float4);
  size_t b_fslots = size_t(m->fine_nslots) * sizeof(Slot);
  if ((e = hipMalloc(&m->slots_d, b_slots)) != hipSuccess) return fail(e, "hipMalloc slots");
  if ((e = hipMalloc(&m->vox_count, b_cnt)) != hipSuccess) return fail(e, "hipMalloc counts");
  if ((e = hipMalloc(&m->vox_key, b_key)) != hipSuccess) return fail(e, "hipMalloc keys");
  if ((e = hipMalloc(&m->vox_pts, b_pts)) != hipSuccess) return fail(e, "hipMalloc points");
  if ((e = hipMalloc(&m->cov, b_cov)) != hipSuccess) return fail(e, "hipMalloc cov");
  if ((e = hipMalloc(&m->vox_cov, b_vcov)) != hipSuccess) return fail(e, "hipMalloc cov");
  if ((e = hipMalloc(&m->vox_nbr, b_nbr)) != hipSuccess) return fail(e, "hipMalloc nbr");
  if ((e = hipMalloc(&m->pt_xyz, b_xyz)) != hipSuccess) return fail(e, "hipMalloc xyz");
  if ((e = hipMalloc(&m->pt_loc, b_loc)) != hipSuccess) return fail(e, "hipMalloc loc");
  if ((e = hipMalloc(&m->vox_slot, b_vslot)) != hipSuccess) return fail(e, "hipMalloc vslot");
  if ((e = hipMalloc(&m->cert, b_cert)) != hipSuccess) return fail(e, "hipMalloc cert");
  if ((e = hipMalloc(&m->cert_mark, b_mark)) != hipSuccess) return fail(e, "hipMalloc mark");
  if ((e = hipMalloc(&m->gslots, b_gslots)) != hipSuccess) return fail(e, "hipMalloc ghosts");
  if ((e = hipMalloc(&m->gkey, b_gkey)) != hipSuccess) return fail(e, "hipMalloc ghosts");
  if ((e = hipMalloc(&m->gnbr, b_gnbr)) != hipSuccess) return fail(e, "hipMalloc ghosts");
  if ((e = hipMalloc(&m->gcount, sizeof(uint32_t))) != hipSuccess) return fail(e, "hipMalloc ghosts");
  if ((e = hipMalloc(&m->fine_pts, b_fpts)) != hipSuccess) return fail(e, "hipMalloc fine");
  if ((e = hipMalloc(&m->fine_slots, b_fslots)) != hipSuccess) return fail(e, "hipMalloc fine");
  m->bytes = int64_t(b_slots + b_cnt + b_key + b_pts + b_cov + b_vcov + b_nbr + b_xyz + b_loc + b_vslot +
                     b_cert + b_mark + b_gslots + b_gkey + b_gnbr + sizeof(uint32_t) + b_fpts +
                     b_fslots);
  if ((e = hipMemsetAsync(m->slots_d, 0xFF, b_slots, st)) != hipSuccess) return fail(e, "memset");
  if ((e = hipMemsetAsync(m->vox_count, 0, b_cnt, st)) != hipSuccess) return fail(e, "memset");
  if ((e = hipMemsetAsync(m->cert_mark, 0, b_mark, st)) != hipSuccess) return fail(e, "memset");
  if ((e = hipMemsetAsync(m->gslots, 0xFF, b_gslots, st)) != hipSuccess) return fail(e, "memset");
  if ((e = hipMemsetAsync(m->gcount, 0, sizeof(uint32_t), st)) != hipSuccess)
    return fail(e, "memset");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "sync");
  *out = m;
  return FAR_OK;
}

far_status_t far_map_destroy(far_map_t m) {
  if (!m) return FAR_OK;
  hipError_t e = hipDeviceSynchronize();
  free_ws(m->ws);
  m->ws = nullptr;
  void* ptrs[] = {m->slots_d, m->vox_count, m->vox_key, m->vox_pts, m->cov, m->vox_cov,
                  m->vox_nbr, m->pt_xyz,
                  m->pt_loc, m->vox_slot, m->cert, m->cert_mark, m->gslots, m->gkey,
                  m->gnbr, m->gcount, m->fine_pts, m->fine_slots};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize", __FILE__, __LINE__);
  return FAR_OK;
}

far_status_t far_map_insert(far_map_t m, const float* xyz, int64_t n, const int32_t* caps,
                            far_stream_t stream, int64_t* n_accepted) {
  if (n_accepted) *n_accepted = 0;
  if (!m || n < 0 || n >= (int64_t(1) << 31) || (n > 0 && !xyz)) {
    set_error("far_map_insert: invalid argument");
    return FAR_E_INVALID;
  }
  if (n == 0) return FAR_OK;
  hipStream_t st = S(stream);
  Scratch scr(st);
  Runs r;
  FAR_TRY(build_runs(xyz, n, m->p.voxel_size, st, scr, r));
  m->fine_ok = false;
  MapView mv = m->view();
  int32_t* seg_vox;
  uint32_t *is_new, *new_rank;
  FAR_TRY(scr.get(&seg_vox, size_t(n)));
  FAR_TRY(scr.get(&is_new, size_t(n)));
  FAR_TRY(scr.get(&new_rank, size_t(n)));
  k_seg_lookup<<<blocks_for(n), kT, 0, st>>>(mv, r.keys, r.seg_start, r.counters + 2, n,
                                             seg_vox, is_new);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(is_new, new_rank, n, r.counters + 3, st, scr));
  uint32_t h_cnt[4];
  FAR_HIP(hipMemcpyAsync(h_cnt, r.counters, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  const int64_t n_seg = h_cnt[2], n_new = h_cnt[3];
  if (h_cnt[1] > 0) {
    set_error("far_map_insert: %u points have voxel keys outside [-2^20, 2^20)", h_cnt[1]);
    return FAR_E_INVALID;
  }
  if (m->n_voxels + n_new > m->voxel_cap) {
    set_error("far_map_insert: %lld new voxels exceed the voxel capacity %lld",
              (long long)n_new, (long long)m->voxel_cap);
    return FAR_E_CAPACITY;
  }
  if (n_seg == 0) return FAR_OK;
  k_seg_claim<<<blocks_for(n_seg), kT, 0, st>>>(m->slots_d, uint32_t(m->slots - 1),
                                                m->log2_slots, r.keys, r.seg_start, is_new,
                                                new_rank, n_seg, m->n_voxels, seg_vox,
                                                m->vox_key, m->vox_slot);
  FAR_HIP(hipGetLastError());
  uint32_t *acc_flag, *id_local, *acc_total;
  int32_t *acc_pos, *seg_newcount;
  FAR_TRY(scr.get(&acc_flag, size_t(n)));
  FAR_TRY(scr.get(&id_local, size_t(n)));
  FAR_TRY(scr.get(&acc_pos, size_t(n)));
  FAR_TRY(scr.get(&seg_newcount, size_t(n_seg)));
  FAR_TRY(scr.get(&acc_total, 1));
  FAR_HIP(hipMemsetAsync(acc_flag, 0, size_t(n) * sizeof(uint32_t), st));
  double dmin2 = m->dmin > 0 ? m->dmin * m->dmin : 0.0;
  k_greedy<<<blocks_for(n_seg), kT, 0, st>>>(xyz, n, caps, m->p.max_pts_per_voxel, dmin2,
                                             r.vals, r.seg_start, r.seg_end, n_seg, seg_vox,
                                             m->vox_count, m->vox_pts, acc_flag, acc_pos,
                                             seg_newcount);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(acc_flag, id_local, n, acc_total, st, scr));
  uint32_t h_acc = 0;
  FAR_HIP(hipMemcpyAsync(&h_acc, acc_total, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  int64_t room = m->p.point_capacity - m->n_points;
  int64_t n_commit = int64_t(h_acc) < room ? int64_t(h_acc) : room;
  bool truncated = int64_t(h_acc) > n_commit;
  k_commit<<<blocks_for(n), kT, 0, st>>>(xyz, n, acc_flag, id_local, acc_pos, m->n_points,
                                         m->p.point_capacity, m->vox_pts, m->pt_xyz,
                                         m->pt_loc);
  FAR_HIP(hipGetLastError());
  uint32_t* seg_changed;
  FAR_TRY(scr.get(&seg_changed, size_t(n_seg)));
  k_counts<<<blocks_for(n_seg), kT, 0, st>>>(n_seg, seg_vox, seg_newcount, truncated, r.vals,
                                             r.seg_start, r.seg_end, acc_flag, id_local,
                                             n_commit, m->vox_count, m->vox_slot,
                                             m->slots_d, seg_changed);
  FAR_HIP(hipGetLastError());
  k_nbr_update<<<blocks_for(n_seg), kT, 0, st>>>(m->view(), n_seg, seg_vox, is_new, m->vox_key,
                                                 m->vox_count, m->vox_nbr);
  FAR_HIP(hipGetLastError());
  // certificates of the points within v of an added point
  if (++m->cert_gen == 0) {
    FAR_HIP(hipMemsetAsync(m->cert_mark, 0, size_t(m->voxel_cap) * sizeof(uint32_t), st));
    m->cert_gen = 1;
  }
  k_cert_mark<<<blocks_for(n_seg), kT, 0, st>>>(n_seg, seg_vox, seg_changed, m->vox_nbr,
                                                m->cert_mark, m->cert_gen);
  FAR_HIP(hipGetLastError());
  {
    const int64_t nv = m->n_voxels + n_new;
    k_cert_build<<<blocks_for(nv * m->p.max_pts_per_voxel), kT, 0, st>>>(
        m->view(), nv, m->cert_mark, m->cert_gen, m->cert);
    FAR_HIP(hipGetLastError());
  }
  FAR_TRY(ghosts_update(m, n_seg, seg_vox, is_new, seg_changed, n_new, st));
  FAR_TRY(map_covariances(m->view(), m->cov, m->n_points, m->n_points + n_commit,
                          m->p.k_cov, st));
  if (n_commit > 0) {
    k_vox_cov<<<blocks_for(n_commit), kT, 0, st>>>(m->cov, m->pt_loc, m->n_points,
                                                   m->n_points + n_commit, m->vox_cov);
    FAR_HIP(hipGetLastError());
  }
  m->n_points += n_commit;
  m->n_voxels += n_new;
  if (n_accepted) *n_accepted = n_commit;
  FAR_HIP(hipStreamSynchronize(st));
  if (truncated) {
    set_error("far_map_insert: point capacity %lld reached; %lld accepted points dropped",
              (long long)m->p.point_capacity, (long long)(int64_t(h_acc) - n_commit));
    return FAR_E_CAPACITY;
  }
  return FAR_OK;
}

far_status_t far_map_knn(far_map_t m, const float* q, int64_t n, int32_t k, double radius,
                         int32_t* idx, float* d2, int32_t* count, far_stream_t stream) {
  if (!m || n < 0 || k < 1 || k > 32 || !(radius > 0.0) || radius > m->p.voxel_size ||
      (n > 0 && (!q || !idx))) {
    set_error("far_map_knn: invalid argument (need 1 <= k <= 32, 0 < radius <= v)");
    return FAR_E_INVALID;
  }
  if (n == 0) return FAR_OK;
  hipStream_t st = S(stream);
  MapView mv = m->view();
  double r2 = radius * radius;
  return dispatch_k(k, [&](auto KK) -> far_status_t {
    constexpr int K = decltype(KK)::value;
    k_map_knn<K><<<blocks_for(n), kT, 0, st>>>(mv, q, n, k, r2, idx, d2, count);
    FAR_HIP(hipGetLastError());
    return FAR_OK;
  });
}

// Voxel grid of a batch of scans with cells of edge `cell` (points grouped by
// scan, then by cell key): sorted points, runs and a hash of the runs.
// *oor receives the number of points whose cell key is out of range (the
// grid is then not built).
// The runs of a scan grid sorted by (scan, key) through compact keys (see
// k_key_range), and each run by x up to 2^-*fb_out cells (*fb_out = 0: runs
// unordered).  *used = false when the batch has no finite point or its key
// range needs more than 62 bits with the scan id; *oor receives the points
// whose keys leave [-2^20, 2^20) (nothing else is done then).
static far_status_t build_runs_compact(const float* xyz, const int64_t* offsets, int32_t S_,
                                       int64_t n, double cell, hipStream_t st, Scratch& scr,
                                       Runs& r, uint32_t** sid_out, bool* used, uint32_t* oor,
                                       int* fb_out) {
  *used = false;
  *oor = 0;
  *fb_out = 0;
  const int64_t nb = (n + int64_t(kT) * kRangePts - 1) / (int64_t(kT) * kRangePts);
  int32_t *part, *rng;
  uint32_t* part_oor;
  FAR_TRY(scr.get(&part, size_t(nb) * 6));
  FAR_TRY(scr.get(&part_oor, size_t(nb)));
  FAR_TRY(scr.get(&rng, 7));
  int e2 = 0;
  const int32_t pow2 = std::frexp(cell, &e2) == 0.5 ? 1 : 0;
  k_key_range<<<unsigned(nb), kT, 0, st>>>(xyz, n, cell, 1.0 / cell, pow2, part, part_oor);
  FAR_HIP(hipGetLastError());
  k_key_range_final<<<1, kT, 0, st>>>(part, part_oor, nb, rng);
  FAR_HIP(hipGetLastError());
  int32_t h[7];
  FAR_HIP(hipMemcpyAsync(h, rng, sizeof(h), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  *oor = uint32_t(h[6]);
  if (h[6] > 0 || h[0] > h[3]) return FAR_OK;
  CompactKey ck;
  ck.mx = h[0];
  ck.my = h[1];
  ck.mz = h[2];
  ck.bx = std::max(ceil_log2(int64_t(h[3]) - h[0] + 1), 2);
  ck.by = std::max(ceil_log2(int64_t(h[4]) - h[1] + 1), 2);
  ck.bz = std::max(ceil_log2(int64_t(h[5]) - h[2] + 1), 2);
  ck.kb = ck.bx + ck.by + ck.bz;
  const int key_bits = (S_ > 1 ? ceil_log2(S_) : 0) + ck.kb + 1;
  if (key_bits > 62) return FAR_OK;
  // x bits: one more radix pass of 8 bits (8 to 15 bits), within 62 in all
  ck.fb = std::min(((key_bits + 15) / 8) * 8 - key_bits, 62 - key_bits);
  const int bits = key_bits + ck.fb;
  uint64_t *ckeys, *ckeys_alt;
  uint32_t* vals_alt;
  FAR_TRY(scr.get(&ckeys, size_t(n)));
  FAR_TRY(scr.get(&ckeys_alt, size_t(n)));
  FAR_TRY(scr.get(&r.keys, size_t(n)));
  FAR_TRY(scr.get(&r.vals, size_t(n)));
  FAR_TRY(scr.get(&vals_alt, size_t(n)));
  FAR_TRY(scr.get(&r.head, size_t(n)));
  FAR_TRY(scr.get(&r.head_scan, size_t(n)));
  FAR_TRY(scr.get(&r.seg_start, size_t(n)));
  FAR_TRY(scr.get(&r.seg_end, size_t(n)));
  FAR_TRY(scr.get(&r.counters, 4));
  uint32_t* sid = nullptr;
  if (S_ > 1) FAR_TRY(scr.get(&sid, size_t(n)));
  FAR_HIP(hipMemsetAsync(r.counters, 0, 4 * sizeof(uint32_t), st));
  k_keys_compact<<<blocks_for(n), kT, 0, st>>>(xyz, n, cell, 1.0 / cell, pow2,
                                                S_ > 1 ? offsets : nullptr, S_, ck, ckeys,
                                                r.vals);
  FAR_HIP(hipGetLastError());
  bool alt = false;
  FAR_TRY(radix_sort_pairs(ckeys, r.vals, ckeys_alt, vals_alt, n, bits, st, scr, &alt));
  if (alt) r.vals = vals_alt;
  k_keys_expand<<<blocks_for(n), kT, 0, st>>>(alt ? ckeys_alt : ckeys, n, ck, r.keys, sid);
  FAR_HIP(hipGetLastError());
  k_grid_heads<<<blocks_for(n), kT, 0, st>>>(r.keys, sid, n, r.head);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(r.head, r.head_scan, n, r.counters + 2, st, scr));
  k_grid_bounds<<<blocks_for(n), kT, 0, st>>>(r.keys, sid, n, r.head, r.head_scan,
                                              r.seg_start, r.seg_end);
  FAR_HIP(hipGetLastError());
  *sid_out = sid;
  *used = true;
  *fb_out = ck.fb;
  return FAR_OK;
}

static far_status_t build_grid(const float* xyz, const int64_t* offsets, int32_t S_, int64_t n,
                               double v, double cell, hipStream_t st, Scratch& scr,
                               GridView* out, uint32_t* oor, uint32_t* order = nullptr,
                               float4* sorted_in = nullptr) {
  Runs r;
  uint32_t* sid = nullptr;
  bool compact = false;
  int fb = 0;
  FAR_TRY(build_runs_compact(xyz, offsets, S_, n, cell, st, scr, r, &sid, &compact, oor, &fb));
  if (*oor > 0) return FAR_OK;
  if (!compact) FAR_TRY(build_runs(xyz, n, cell, st, scr, r));
  uint64_t* keys = r.keys;
  uint32_t* vals = r.vals;
  if (S_ > 1 && !compact) {
    // second stable sort, by scan id, keeps the key order inside every scan
    uint64_t *sid_key, *sid_alt, *keys2;
    uint32_t *perm, *perm_alt, *vals2;
    FAR_TRY(scr.get(&sid_key, size_t(n)));
    FAR_TRY(scr.get(&sid_alt, size_t(n)));
    FAR_TRY(scr.get(&perm, size_t(n)));
    FAR_TRY(scr.get(&perm_alt, size_t(n)));
    FAR_TRY(scr.get(&keys2, size_t(n)));
    FAR_TRY(scr.get(&vals2, size_t(n)));
    FAR_TRY(scr.get(&sid, size_t(n)));
    k_scan_ids<<<blocks_for(n), kT, 0, st>>>(r.vals, n, offsets, S_, sid_key, perm);
    FAR_HIP(hipGetLastError());
    FAR_TRY(radix_sort_pairs(sid_key, perm, sid_alt, perm_alt, n, ceil_log2(S_), st, scr));
    k_apply_perm<<<blocks_for(n), kT, 0, st>>>(perm, n, r.keys, r.vals, keys2, vals2,
                                               sid_key, sid);
    FAR_HIP(hipGetLastError());
    keys = keys2;
    vals = vals2;
    k_grid_heads<<<blocks_for(n), kT, 0, st>>>(keys, sid, n, r.head);
    FAR_HIP(hipGetLastError());
    FAR_TRY(scan_exclusive(r.head, r.head_scan, n, r.counters + 2, st, scr));
    k_grid_bounds<<<blocks_for(n), kT, 0, st>>>(keys, sid, n, r.head, r.head_scan,
                                                r.seg_start, r.seg_end);
    FAR_HIP(hipGetLastError());
  }
  if (!compact) {   // keys out of range are found by the full-key pass only
    uint32_t h_cnt[4];
    FAR_HIP(hipMemcpyAsync(h_cnt, r.counters, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
    FAR_HIP(hipStreamSynchronize(st));
    *oor = h_cnt[1];
    if (h_cnt[1] > 0) return FAR_OK;
  }
  // The number of runs stays on the device (r.counters[2]): the kernels below
  // are launched for one run per point and read it.
  // two slots per point, each scan's in its own stretch (n < 2^31)
  const int64_t n_slots = 2 * n;
  Slot* slots;
  float4* sorted;
  FAR_TRY(scr.get(&slots, size_t(n_slots)));
  if (sorted_in)
    sorted = sorted_in;   // the caller's packed A words: the sorted points are exactly those
  else
    FAR_TRY(scr.get(&sorted, size_t(n)));
  FAR_HIP(hipMemsetAsync(slots, 0xFF, size_t(n_slots) * sizeof(Slot), st));
  k_gather_sorted<<<unsigned(((blocks_for(n) + 7) / 8) * 8), kT, 0, st>>>(xyz, n, vals, sorted,
                                                                        order);
  FAR_HIP(hipGetLastError());
  int e2 = 0;
  const int32_t pow2 = std::frexp(cell, &e2) == 0.5 ? 1 : 0;
  // a later point of an x-sorted run lies at most one quantum (2^-fb cells,
  // plus the rounding of x / cell) below an earlier one; twice that is kept
  const double mx = compact && fb > 0 ? std::ldexp(cell, 1 - fb) : HUGE_VAL;
  uint2* nbt;
  FAR_TRY(scr.get(&nbt, size_t(n) * 27));
  *out = GridView{slots, sorted, keys, sid, r.seg_start, r.seg_end, v, cell, 1.0 / cell, pow2,
                  S_ > 1 ? offsets : nullptr, uint32_t(n_slots), mx, r.head, r.head_scan,
                  nbt, r.counters + 2, nullptr, nullptr};
  k_grid_claim<<<kGridBlocks, kT, 0, st>>>(*out, slots);
  FAR_HIP(hipGetLastError());
  k_grid_nbr_table<<<kGridBlocks, kT, 0, st>>>(*out, nbt);
  FAR_HIP(hipGetLastError());
  return FAR_OK;
}

// Points per voxel run from which the covariance search takes one wave per
// run (k_grid_cov_wave) instead of one lane per point; 0 = never.
static int32_t g_dense_threshold = 0;

static far_status_t scan_cov_impl(const float* xyz, const int64_t* offsets, int32_t S_,
                                  int64_t n, double voxel_size, int32_t k, float* cov6,
                                  uint8_t* valid, hipStream_t st, const char* who,
                                  uint32_t* order = nullptr, void* packed = nullptr) {
  Scratch scr(st);
  TimedScope ts(FAR_TIME_COVARIANCES, st);
  GridView g{};
  uint32_t oor = 0;
  char* pk = static_cast<char*>(packed);
  FAR_TRY(build_grid(xyz, offsets, S_, n, voxel_size, voxel_size, st, scr, &g, &oor, order,
                     reinterpret_cast<float4*>(pk)));
  if (pk) {
    g.pk_B = reinterpret_cast<float4*>(pk + 16 * n);
    g.pk_C = reinterpret_cast<float2*>(pk + 32 * n);
  }
  if (oor > 0) {
    set_error("%s: %u points have voxel keys outside [-2^20, 2^20)", who, oor);
    return FAR_E_INVALID;
  }
  const int32_t dense = g_dense_threshold;
  // (a batch with no finite point has no runs: every point takes the
  // non-finite branch of k_grid_cov, zero covariance and invalid)
  return dispatch_k(k, [&](auto KK) -> far_status_t {
    constexpr int K = decltype(KK)::value;
    const int64_t cov_grid = ((blocks_for(n) + 7) / 8) * 8;
    k_grid_cov<K><<<unsigned(cov_grid), kT, 0, st>>>(g, dense, n, k, g_cov_reg, cov6, valid);
    FAR_HIP(hipGetLastError());
    if (dense > 0) {   // a persistent grid of 64 waves per CU over the runs
      k_grid_cov_wave<K><<<256 * 64, 64, 0, st>>>(g, dense, n, k, g_cov_reg, cov6, valid);
      FAR_HIP(hipGetLastError());
    }
    return FAR_OK;
  });
}

far_status_t far_scan_covariances(const float* xyz, int64_t n, double voxel_size, int32_t k,
                                  float* cov6, uint8_t* valid, far_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !(voxel_size > 0.0) || k < 1 || k > 32 ||
      (n > 0 && (!xyz || !cov6 || !valid))) {
    set_error("far_scan_covariances: invalid argument");
    return FAR_E_INVALID;
  }
  if (n == 0) return FAR_OK;
  return scan_cov_impl(xyz, nullptr, 1, n, voxel_size, k, cov6, valid, S(stream),
                       "far_scan_covariances");
}

far_status_t far_scan_covariances_batch(const float* xyz, const int64_t* offsets, int32_t S_,
                                        int64_t n_total, double voxel_size, int32_t k,
                                        float* cov6, uint8_t* valid, far_stream_t stream) {
  if (S_ < 1 || !offsets || n_total < 0 || n_total >= (int64_t(1) << 31) ||
      !(voxel_size > 0.0) || k < 1 || k > 32 || (n_total > 0 && (!xyz || !cov6 || !valid))) {
    set_error("far_scan_covariances_batch: invalid argument");
    return FAR_E_INVALID;
  }
  if (n_total == 0) return FAR_OK;
  return scan_cov_impl(xyz, offsets, S_, n_total, voxel_size, k, cov6, valid, S(stream),
                       "far_scan_covariances_batch");
}

far_status_t far_scan_covariances_batch_order(const float* xyz, const int64_t* offsets,
                                              int32_t S_, int64_t n_total, double voxel_size,
                                              int32_t k, float* cov6, uint8_t* valid,
                                              uint32_t* order, far_stream_t stream) {
  if (S_ < 1 || !offsets || n_total < 0 || n_total >= (int64_t(1) << 31) ||
      !(voxel_size > 0.0) || k < 1 || k > 32 ||
      (n_total > 0 && (!xyz || !cov6 || !valid || !order))) {
    set_error("far_scan_covariances_batch_order: invalid argument");
    return FAR_E_INVALID;
  }
  if (n_total == 0) return FAR_OK;
  return scan_cov_impl(xyz, offsets, S_, n_total, voxel_size, k, cov6, valid, S(stream),
                       "far_scan_covariances_batch_order", order);
}

far_status_t far_scan_covariances_batch_packed(const float* xyz, const int64_t* offsets,
                                               int32_t S_, int64_t n_total, double voxel_size,
                                               int32_t k, float* cov6, uint8_t* valid,
                                               void* packed, far_stream_t stream) {
  if (S_ < 1 || !offsets || n_total < 0 || n_total >= (int64_t(1) << 31) ||
      !(voxel_size > 0.0) || k < 1 || k > 32 ||
      (n_total > 0 && (!xyz || !cov6 || !valid || !packed)) ||
      (reinterpret_cast<uintptr_t>(packed) & 15) != 0) {
    set_error("far_scan_covariances_batch_packed: invalid argument");
    return FAR_E_INVALID;
  }
  if (n_total == 0) return FAR_OK;
  return scan_cov_impl(xyz, offsets, S_, n_total, voxel_size, k, cov6, valid, S(stream),
                       "far_scan_covariances_batch_packed", nullptr, packed);
}

far_status_t far_voxel_downsample(const float* xyz, int64_t n, double v, float* out,
                                  int32_t* keep, int64_t* n_out, far_stream_t stream) {
  if (n_out) *n_out = 0;
  if (!n_out || n < 0 || n >= (int64_t(1) << 31) || !(v > 0.0) || !std::isfinite(v) ||
      (n > 0 && (!xyz || !out)) || (n > 0 && out == xyz)) {
    set_error("far_voxel_downsample: invalid argument");
    return FAR_E_INVALID;
  }
  if (n == 0) return FAR_OK;
  hipStream_t st = S(stream);
  Scratch scr(st);
  Runs r;
  FAR_TRY(build_runs(xyz, n, v, st, scr, r));
  uint32_t *flag, *pos, *total;
  FAR_TRY(scr.get(&flag, size_t(n)));
  FAR_TRY(scr.get(&pos, size_t(n)));
  FAR_TRY(scr.get(&total, 1));
  k_ds_flags<<<blocks_for(n), kT, 0, st>>>(r.vals, r.head, n, flag);
  FAR_HIP(hipGetLastError());
  FAR_TRY(scan_exclusive(flag, pos, n, total, st, scr));
  uint32_t h[2];
  FAR_HIP(hipMemcpyAsync(&h[0], r.counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipMemcpyAsync(&h[1], total, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  if (h[0] > 0) {
    set_error("far_voxel_downsample: %u points have voxel keys outside [-2^20, 2^20)", h[0]);
    return FAR_E_INVALID;
  }
  const int64_t m = h[1];
  if (m > 0) {
    k_ds_scatter<<<blocks_for(n), kT, 0, st>>>(xyz, n, flag, pos, m, out, keep);
    FAR_HIP(hipGetLastError());
  }
  FAR_HIP(hipStreamSynchronize(st));
  *n_out = m;
  return FAR_OK;
}

far_status_t far_transform_points(const float* xyz, int64_t n, const double T[16], float* out,
                                  far_stream_t stream) {
  if (n < 0 || !T || (n > 0 && (!xyz || !out))) {
    set_error("far_transform_points: invalid argument");
    return FAR_E_INVALID;
  }
  Rigid R;
  for (int i = 0; i < 12; ++i) {
    R.r[i] = T[i];
    if (!std::isfinite(T[i])) {
      set_error("far_transform_points: non-finite pose");
      return FAR_E_INVALID;
    }
  }
  if (n == 0) return FAR_OK;
  k_transform<<<blocks_for(n), kT, 0, S(stream)>>>(xyz, n, R, out);
  FAR_HIP(hipGetLastError());
  return FAR_OK;
}

far_status_t far_set_covariance_schedule(int32_t dense_threshold) {
  if (dense_threshold < 0) {
    set_error("far_set_covariance_schedule: dense_threshold must be >= 0");
    return FAR_E_INVALID;
  }
  g_dense_threshold = dense_threshold;
  return FAR_OK;
}

far_status_t far_set_covariance_regularisation(int32_t mode) {
  if (mode != FAR_REG_EQ1 && mode != FAR_REG_PLANE) {
    set_error("far_set_covariance_regularisation: unknown mode %d", mode);
    return FAR_E_INVALID;
  }
  g_cov_reg = mode;
  return FAR_OK;
}

far_status_t far_get_covariance_regularisation(int32_t* mode) {
  if (!mode) {
    set_error("far_get_covariance_regularisation: null argument");
    return FAR_E_INVALID;
  }
  *mode = g_cov_reg;
  return FAR_OK;
}

far_status_t far_get_covariance_schedule(int32_t* dense_threshold) {
  if (!dense_threshold) {
    set_error("far_get_covariance_schedule: null argument");
    return FAR_E_INVALID;
  }
  *dense_threshold = g_dense_threshold;
  return FAR_OK;
}

far_status_t far_autotune_covariances(const float* xyz, const int64_t* offsets, int32_t S_,
                                      int64_t n_total, double voxel_size, int32_t k,
                                      float* cov6, uint8_t* valid, int32_t reps, int32_t* best,
                                      double* ms, far_stream_t stream) {
  if (!best || reps < 1 || reps > 100) {
    set_error("far_autotune_covariances: invalid argument");
    return FAR_E_INVALID;
  }
  hipStream_t st = S(stream);
  const int32_t saved = g_dense_threshold;
  const int32_t cands[5] = {0, 16, 32, 64, 128};
  double times[5];
  int32_t win = saved;
  double win_ms = -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  far_status_t rs = FAR_OK;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    rs = hip_fail(e, "far_autotune_covariances setup", __FILE__, __LINE__);
  for (int c = 0; c < 5 && rs == FAR_OK; ++c) {
    g_dense_threshold = cands[c];
    double bestc = 1e300;
    for (int r = 0; r <= reps && rs == FAR_OK; ++r) {
      if ((e = hipEventRecord(e0, st)) != hipSuccess) {
        rs = hip_fail(e, "far_autotune_covariances", __FILE__, __LINE__);
        break;
      }
      rs = far_scan_covariances_batch(xyz, offsets, S_, n_total, voxel_size, k, cov6, valid,
                                      stream);
      if (rs != FAR_OK) break;
      float t = 0.0f;
      if ((e = hipEventRecord(e1, st)) != hipSuccess ||
          (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
        rs = hip_fail(e, "far_autotune_covariances timing", __FILE__, __LINE__);
        break;
      }
      if (r > 0 && t < bestc) bestc = t;
    }
    times[c] = bestc;
    if (rs == FAR_OK && (win_ms < 0.0 || bestc < win_ms)) {
      win_ms = bestc;
      win = cands[c];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rs != FAR_OK) {
    g_dense_threshold = saved;
    return rs;
  }
  // the threshold in place stays unless a candidate beats it by more than 2 %
  for (int c = 0; c < 5; ++c)
    if (cands[c] == saved && times[c] <= 1.02 * win_ms) win = saved;
  g_dense_threshold = win;
  *best = win;
  if (ms)
    for (int c = 0; c < 5; ++c) ms[c] = times[c];
  return FAR_OK;
}

far_status_t far_asmd_caps(const float* xyz_sensor, const float* xyz_map, int64_t n, double v,
                           int32_t k, int32_t nmax, double r_near, double r_max, int32_t* caps,
                           double* mean_near, far_stream_t stream) {
  if (n < 0 || n >= (int64_t(1) << 31) || !(v > 0.0) || !std::isfinite(v) || k < 1 ||
      nmax < k || nmax > 64 || !(r_near >= 0.0) || !(r_max > 0.0) ||
      (n > 0 && (!xyz_sensor || !xyz_map || !caps))) {
    set_error("far_asmd_caps: invalid argument");
    return FAR_E_INVALID;
  }
  double mean = double(nmax);
  if (n > 0) {
    hipStream_t st = S(stream);
    Scratch scr(st);
    const int set_log2 = std::max(6, ceil_log2(2 * n));
    const int64_t set_n = int64_t(1) << set_log2;
    uint64_t* set;
    uint32_t* counters;
    FAR_TRY(scr.get(&set, size_t(set_n)));
    FAR_TRY(scr.get(&counters, 3));
    {
      TimedScope ts(FAR_TIME_ASMD, st);
      FAR_HIP(hipMemsetAsync(set, 0xFF, size_t(set_n) * sizeof(uint64_t), st));
      FAR_HIP(hipMemsetAsync(counters, 0, 3 * sizeof(uint32_t), st));
      k_asmd_count<<<blocks_for(n), kT, 0, st>>>(xyz_sensor, xyz_map, n, v, r_near * r_near,
                                                 set, uint32_t(set_n - 1), set_log2, counters);
      FAR_HIP(hipGetLastError());
      k_asmd_caps<<<blocks_for(n), kT, 0, st>>>(xyz_sensor, n, counters, r_max, k, nmax, caps);
      FAR_HIP(hipGetLastError());
    }
    uint32_t h[3];
    FAR_HIP(hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, st));
    FAR_HIP(hipStreamSynchronize(st));
    if (h[2] > 0) {
      set_error("far_asmd_caps: %u near points have voxel keys outside [-2^20, 2^20)", h[2]);
      return FAR_E_INVALID;
    }
    if (h[1] > 0) mean = double(h[0]) / double(h[1]);
  }
  if (mean_near) *mean_near = mean;
  return FAR_OK;
}

far_status_t far_map_evict(far_map_t m, const double c[3], double radius, int64_t* n_removed,
                           far_stream_t stream) {
  if (n_removed) *n_removed = 0;
  if (!m || !c || !(radius >= 0.0) || !std::isfinite(c[0]) || !std::isfinite(c[1]) ||
      !std::isfinite(c[2])) {
    set_error("far_map_evict: invalid argument");
    return FAR_E_INVALID;
  }
  const int64_t n = m->n_points;
  hipStream_t st = S(stream);
  const double v = m->p.voxel_size;
  if (n == 0) {
    // only empty voxels can be held: drop them too (the map is rebuilt from
    // its surviving points)
    if (m->n_voxels > 0) {
      FAR_HIP(hipMemsetAsync(m->slots_d, 0xFF, size_t(m->slots) * sizeof(Slot), st));
      FAR_HIP(hipMemsetAsync(m->vox_count, 0, size_t(m->n_voxels) * sizeof(int32_t), st));
      FAR_TRY(ghosts_reset(m, st));
      FAR_HIP(hipStreamSynchronize(st));
      m->n_voxels = 0;
      m->fine_ok = false;
    }
    return FAR_OK;
  }
  Scratch scr(st);
  uint32_t *keep, *nid, *total;
  FAR_TRY(scr.get(&keep, size_t(n)));
  FAR_TRY(scr.get(&nid, size_t(n)));
  FAR_TRY(scr.get(&total, 1));
  {
    TimedScope ts(FAR_TIME_EVICT, st);
    k_evict_keep<<<blocks_for(n), kT, 0, st>>>(m->pt_xyz, m->p.point_capacity, n, v, c[0],
                                               c[1], c[2], radius * radius, keep);
    FAR_HIP(hipGetLastError());
    FAR_TRY(scan_exclusive(keep, nid, n, total, st, scr));
  }
  uint32_t h_keep = 0;
  FAR_HIP(hipMemcpyAsync(&h_keep, total, sizeof(h_keep), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  const int64_t n_keep = h_keep;
  if (n_keep == n) return FAR_OK;
  float* xyz;
  float4* cv;
  FAR_TRY(scr.get(&xyz, size_t(3 * std::max<int64_t>(n_keep, 1))));
  FAR_TRY(scr.get(&cv, size_t(2 * std::max<int64_t>(n_keep, 1))));
  TimedScope ts2(FAR_TIME_EVICT, st);
  k_evict_gather<<<blocks_for(n), kT, 0, st>>>(m->pt_xyz, m->cov, m->p.point_capacity, n, keep,
                                               nid, n_keep, xyz, cv);
  FAR_HIP(hipGetLastError());
  // clear the voxel structures, then store the survivors and rebuild them
  FAR_HIP(hipMemsetAsync(m->slots_d, 0xFF, size_t(m->slots) * sizeof(Slot), st));
  FAR_HIP(hipMemsetAsync(m->vox_count, 0, size_t(m->n_voxels) * sizeof(int32_t), st));
  FAR_TRY(ghosts_reset(m, st));
  m->n_points = 0;
  m->n_voxels = 0;
  m->fine_ok = false;
  if (n_removed) *n_removed = n - n_keep;
  if (n_keep == 0) {
    ts2.stop();
    FAR_HIP(hipStreamSynchronize(st));
    return FAR_OK;
  }
  k_evict_store<<<blocks_for(n_keep), kT, 0, st>>>(xyz, n_keep, m->p.point_capacity, m->pt_xyz);
  FAR_HIP(hipGetLastError());
  FAR_HIP(hipMemcpyAsync(m->cov, cv, size_t(n_keep) * 2 * sizeof(float4),
                         hipMemcpyDeviceToDevice, st));
  Runs r;
  FAR_TRY(build_runs(xyz, n_keep, v, st, scr, r));
  uint32_t h_cnt[4];
  FAR_HIP(hipMemcpyAsync(h_cnt, r.counters, sizeof(h_cnt), hipMemcpyDeviceToHost, st));
  ts2.stop();
  FAR_HIP(hipStreamSynchronize(st));
  const int64_t n_seg = h_cnt[2];
  TimedScope ts3(FAR_TIME_EVICT, st);
  int32_t* seg_vox;
  uint32_t *is_new, *rank;
  FAR_TRY(scr.get(&seg_vox, size_t(n_seg)));
  FAR_TRY(scr.get(&is_new, size_t(n_seg)));
  FAR_TRY(scr.get(&rank, size_t(n_seg)));
  k_all_new<<<blocks_for(n_seg), kT, 0, st>>>(n_seg, is_new, rank);
  FAR_HIP(hipGetLastError());
  k_seg_claim<<<blocks_for(n_seg), kT, 0, st>>>(m->slots_d, uint32_t(m->slots - 1),
                                                m->log2_slots, r.keys, r.seg_start, is_new, rank,
                                                n_seg, 0, seg_vox, m->vox_key, m->vox_slot);
  FAR_HIP(hipGetLastError());
  k_bulk_place<<<blocks_for(n_keep), kT, 0, st>>>(xyz, n_keep, r.keys, r.vals, r.head,
                                                  r.head_scan, r.seg_start, seg_vox,
                                                  m->p.max_pts_per_voxel, m->vox_pts, m->pt_loc);
  FAR_HIP(hipGetLastError());
  k_bulk_counts<<<blocks_for(n_seg), kT, 0, st>>>(n_seg, r.seg_start, r.seg_end, seg_vox,
                                                  m->vox_slot, m->vox_count, m->slots_d);
  FAR_HIP(hipGetLastError());
  k_nbr_update<<<blocks_for(n_seg), kT, 0, st>>>(m->view(), n_seg, seg_vox, is_new, m->vox_key,
                                                 m->vox_count, m->vox_nbr);
  FAR_HIP(hipGetLastError());
  k_vox_cov<<<blocks_for(n_keep), kT, 0, st>>>(m->cov, m->pt_loc, 0, n_keep, m->vox_cov);
  FAR_HIP(hipGetLastError());
  // every slot changed: all certificates again, and the ghosts
  k_cert_build<<<blocks_for(n_seg * m->p.max_pts_per_voxel), kT, 0, st>>>(
      m->view(), n_seg, nullptr, 0, m->cert);
  FAR_HIP(hipGetLastError());
  FAR_TRY(ghosts_update(m, n_seg, seg_vox, nullptr, nullptr, n_seg, st));
  m->n_points = n_keep;
  m->n_voxels = n_seg;
  ts3.stop();
  FAR_HIP(hipStreamSynchronize(st));
  return FAR_OK;
}

far_status_t far_map_stats(far_map_t m, far_map_stats_t* out, far_stream_t stream) {
  if (!m || !out) {
    set_error("far_map_stats: null argument");
    return FAR_E_INVALID;
  }
  hipStream_t st = S(stream);
  Scratch scr(st);
  unsigned long long* sum;
  uint32_t* maxp;
  FAR_TRY(scr.get(&sum, 1));
  FAR_TRY(scr.get(&maxp, 1));
  FAR_HIP(hipMemsetAsync(sum, 0, sizeof(unsigned long long), st));
  FAR_HIP(hipMemsetAsync(maxp, 0, sizeof(uint32_t), st));
  k_probe_stats<<<blocks_for(m->slots), kT, 0, st>>>(m->slots_d, m->slots,
                                                     uint32_t(m->slots - 1), m->log2_slots,
                                                     sum, maxp);
  FAR_HIP(hipGetLastError());
  unsigned long long h_sum = 0;
  uint32_t h_max = 0;
  FAR_HIP(hipMemcpyAsync(&h_sum, sum, sizeof(h_sum), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipMemcpyAsync(&h_max, maxp, sizeof(h_max), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  out->n_points = m->n_points;
  out->n_voxels = m->n_voxels;
  out->table_slots = m->slots;
  out->load_factor = double(m->n_voxels) / double(m->slots);
  out->mean_probe = m->n_voxels ? double(h_sum) / double(m->n_voxels) : 0.0;
  out->max_probe = int32_t(h_max);
  out->max_pts_per_voxel = m->p.max_pts_per_voxel;
  out->voxel_size = m->p.voxel_size;
  out->min_spacing = m->dmin;
  out->bytes_device = m->bytes;
  return FAR_OK;
}

far_status_t far_map_export(far_map_t m, float* xyz, float* cov6, uint8_t* valid,
                            int64_t capacity, int64_t* n_out, far_stream_t stream) {
  if (!m || !n_out) {
    set_error("far_map_export: null argument");
    return FAR_E_INVALID;
  }
  *n_out = m->n_points;
  if (m->n_points > capacity) {
    set_error("far_map_export: map holds %lld points, buffers hold %lld",
              (long long)m->n_points, (long long)capacity);
    return FAR_E_CAPACITY;
  }
  if (m->n_points == 0) return FAR_OK;
  hipStream_t st = S(stream);
  k_export<<<blocks_for(m->n_points), kT, 0, st>>>(m->cov, m->pt_xyz, m->p.point_capacity,
                                                   m->n_points, xyz, cov6, valid);
  FAR_HIP(hipGetLastError());
  FAR_HIP(hipStreamSynchronize(st));
  return FAR_OK;
}

}  // extern "C"
