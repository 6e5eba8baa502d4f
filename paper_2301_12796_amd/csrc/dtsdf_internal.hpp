// Internal definitions of the Directional-TSDF library (device layout, hash, helpers).
//
// Device layout of a map
//   entries  HashEntry[buckets]     open-addressing spatial hash, linear probing; one entry per
//                                   8^3 block holds the pool index of the block's brick in each
//                                   of the six directions (-1: not allocated).  Sec. 7 keys
//                                   bricks by (x, y, z, D); grouping the six D of a block in one
//                                   32-byte entry lets one probe serve every direction a ray
//                                   sample reads.
//   req      uint32[buckets]        per-entry bit mask of directions requested by the frame
//                                   being integrated (cleared when bricks are assigned)
//   bkey     int4[capacity]         (bx, by, bz, D) of every pool brick
//   geo      [capacity*512]         distance and weight of every voxel, brick-major, voxel l at
//                                   local (l % 8, l / 8 % 8, l / 64); the march reads only
//                                   these.  Plain format: float2 (sdf, w), 8 bytes.  Packed
//                                   formats: one 32-bit word, sdf code in bits 0-15 (float16,
//                                   or int16 q with sdf = q / 32767) and the weight code
//                                   q (w = q^2 / 1024, see weight_code) in bits 16-23,
//                                   4 bytes.
//   rgb      uint32[capacity*512]   r | g << 8 | b << 16 colour code per voxel; in the packed
//                                   formats the colour-weight code sits in bits 24-31
//   wc       float[capacity*512]    colour weight per voxel (plain format only)
//   counters int32[16]              [0] bricks handed out (may overshoot the capacity while a
//                                   frame allocates), [1] dropped requests, [2] hash overflow,
//                                   [3] occupied hash entries, [4..9] bounding box of the
//                                   occupied blocks (min x, y, z, max x, y, z)
//   sub_min  float[capacity*8]      per 4^3 sub-block of a brick: min sdf over its voxels with
//                                   w > 0 (+inf if none); sub-block s = sx | sy << 1 | sz << 2
//   slot_min float[buckets*8]       per hash entry and sub-block: min of sub_min over the
//                                   block's directions
//   brick_neg u64[capacity*16]      per brick, word z, bit x + 8 y: the voxel has w > 0 and
//                                   sdf <= kSkipMin; words 8 + z: the voxel has w > 0
//   block_neg u64[buckets*8]        per hash entry: OR of brick_neg over the block's bricks
//                                   (input of the positive-cell words below)
//
// Render index (updated after every integrate / import): a dense grid over the bounding box
// of the occupied blocks.  288 GB of HBM make a dense block grid affordable for room-scale
// maps (160 bytes per 4 cm block at 5 mm voxels), and it turns every block the ray march
// enters into one round of independent loads (record, cell words and group bytes), with no
// hash probing and no chain of dependent lookups:
//   grid_rec  GridRec[gx*gy*gz]     per block: the six brick indices (-1: not allocated), its
//                                   hash slot (-1: absent block) and the info word: bits 0-7
//                                   sub-block skip bits (bit s set: every cell based in
//                                   sub-block s has all corner values > kSkipMin in every
//                                   direction, so the combined SDF is positive wherever
//                                   defined there and no crossing can end in that
//                                   sub-block), bits 8-10 empty level e of an absent block
//                                   (the aligned cell of 2^e blocks per edge containing it
//                                   holds no present block), bit 15 present
//   grid_cell u64[gx*gy*gz*8]       per block, word z, bit x + 8 y: no corner of the cell
//                                   based at voxel (x, y, z) (corners in the +x/+y/+z
//                                   neighbours included) is non-positive in any direction,
//                                   so every direction defined there interpolates positive
//                                   values and the combined SDF is positive wherever defined
//   grid_group u8[gx*gy*gz*64]      per block and 2x2x2 group of cells (byte gx + 4 gy +
//                                   16 gz): bit D set if direction D has all 8 corners
//                                   observed (w > 0) at some cell of the group; a direction
//                                   whose bit is clear is undefined at every cell of the
//                                   group and contributes nothing there
//   mip      uint8[levels 1..6]     occupancy of the aligned cells of 2^l blocks per edge
//                                   (input of the empty levels)
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dtsdf.h"

namespace dtsdf {

constexpr int kB = 8;
constexpr int kVox = 512;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kKeyBias = 1 << 19;   // block coordinates must lie in [-2^19, 2^19)
constexpr float kSkipMin = 1e-6f;   // margin keeping interpolated values strictly positive
constexpr int64_t kMaxGridBlocks = 1ll << 31;

struct alignas(32) HashEntry {
  uint64_t key;
  int32_t brick[6];
};
static_assert(sizeof(HashEntry) == 32, "hash entries are 32 bytes");

// Render-index record of one grid block (see the layout notes above).
struct alignas(32) GridRec {
  int32_t brick[6];
  uint32_t info;
  int32_t slot;
};
static_assert(sizeof(GridRec) == 32, "grid records are 32 bytes");
constexpr uint32_t kRecPresent = 1u << 15;
constexpr int kMipLevels = 6;   // aligned empty cells up to 64 blocks per edge

__host__ __device__ inline bool key_in_range(int bx, int by, int bz) {
  return bx >= -kKeyBias && bx < kKeyBias && by >= -kKeyBias && by < kKeyBias &&
         bz >= -kKeyBias && bz < kKeyBias;
}

__host__ __device__ inline uint64_t pack_key(int bx, int by, int bz) {
  return (uint64_t)(uint32_t)(bx + kKeyBias) | ((uint64_t)(uint32_t)(by + kKeyBias) << 20) |
         ((uint64_t)(uint32_t)(bz + kKeyBias) << 40);
}

__host__ __device__ inline void unpack_key(uint64_t k, int& bx, int& by, int& bz) {
  bx = (int)(k & 0xFFFFF) - kKeyBias;
  by = (int)((k >> 20) & 0xFFFFF) - kKeyBias;
  bz = (int)((k >> 40) & 0xFFFFF) - kKeyBias;
}

__host__ __device__ inline uint32_t hash_key(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}

// Read-only view of a map, passed by value to kernels.
// Storage formats: 0 plain float, 1 float16 distance + uint8 weights, 2 int16 distance
// (scaled by the truncation) + uint8 weights.  Codes are rounded half to even.
// Weight code of the packed formats: q in 0 .. 255 stands for w = q^2 / 1024 (0 .. 63.5).
// The step between codes, (2 q + 1) / 1024, is 0.02 at w = 0.1 and 0.5 at the top, so that
// carving updates (w_carve = 0.1) and small fusion weights accumulate instead of rounding
// back to the old code.  q = round-half-even(sqrt(1024 w)), decided exactly: 1024 w and the
// rounding boundaries (q + 1/2)^2 = q^2 + q + 1/4 are exact float32 values.
__host__ __device__ inline uint32_t weight_code(float w) {
  const float x = 1024.f * fmaxf(0.f, w);
  int q = (int)fminf(256.f, sqrtf(x));
  while (q > 0 && (float)(q * q) > x) --q;
  while (q < 256 && (float)((q + 1) * (q + 1)) <= x) ++q;
  const float mid = (float)(q * q + q) + 0.25f;
  if (x > mid || (x == mid && (q & 1))) ++q;
  return (uint32_t)(q < 255 ? q : 255);
}

__host__ __device__ inline float weight_decode(uint32_t q) {
  return (float)(q * q) * (1.f / 1024.f);
}

template <int F>
struct Vox;

template <>
struct Vox<0> {
  static constexpr int kGeoBytes = 8;
  __host__ __device__ static void load(const void* g, size_t i, float& s, float& w) {
    const float2 v = static_cast<const float2*>(g)[i];
    s = v.x;
    w = v.y;
  }
  __host__ __device__ static void store(void* g, size_t i, float s, float w) {
    static_cast<float2*>(g)[i] = make_float2(s, w);
  }
  __host__ __device__ static void load_color(const uint32_t* rgb, const float* wc, size_t i,
                                             uint32_t& code, float& w) {
    code = rgb[i];
    w = wc[i];
  }
  __host__ __device__ static void store_color(uint32_t* rgb, float* wc, size_t i, uint32_t code,
                                              float w) {
    rgb[i] = code;
    wc[i] = w;
  }
};

struct VoxPacked {
  static constexpr int kGeoBytes = 4;
  __host__ __device__ static float weight(uint32_t v) { return weight_decode((v >> 16) & 0xFFu); }
  __host__ __device__ static void load_color(const uint32_t* rgb, const float*, size_t i,
                                             uint32_t& code, float& w) {
    const uint32_t v = rgb[i];
    code = v & 0xFFFFFFu;
    w = weight_decode(v >> 24);
  }
  __host__ __device__ static void store_color(uint32_t* rgb, float*, size_t i, uint32_t code,
                                              float w) {
    rgb[i] = (code & 0xFFFFFFu) | (weight_code(w) << 24);
  }
};

template <>
struct Vox<1> : VoxPacked {
  __host__ __device__ static void decode(uint32_t v, float& s, float& w) {
    s = __half2float(__ushort_as_half((unsigned short)(v & 0xFFFFu)));
    w = weight(v);
  }
  __host__ __device__ static void load(const void* g, size_t i, float& s, float& w) {
    decode(static_cast<const uint32_t*>(g)[i], s, w);
  }
  __host__ __device__ static void store(void* g, size_t i, float s, float w) {
    static_cast<uint32_t*>(g)[i] =
        (uint32_t)__half_as_ushort(__float2half_rn(s)) | (weight_code(w) << 16);
  }
};

template <>
struct Vox<2> : VoxPacked {
  __host__ __device__ static void decode(uint32_t v, float& s, float& w) {
    s = (float)(int16_t)(v & 0xFFFFu) * (1.0f / 32767.0f);
    w = weight(v);
  }
  __host__ __device__ static void load(const void* g, size_t i, float& s, float& w) {
    decode(static_cast<const uint32_t*>(g)[i], s, w);
  }
  __host__ __device__ static void store(void* g, size_t i, float s, float w) {
    const float q = fminf(32767.f, fmaxf(-32767.f, rintf(s * 32767.f)));
    static_cast<uint32_t*>(g)[i] = (uint32_t)(uint16_t)(int16_t)q | (weight_code(w) << 16);
  }
};

// Kernel instantiation tag of a regular volume (written by dtsdf_combine): plain storage,
// one volume in direction slot 0, rendered without direction weighting.
constexpr int kRegularVolume = 3;
template <>
struct Vox<kRegularVolume> : Vox<0> {};

inline int storage_format(const dtsdf_params& p) {
  if (p.sdf_fmt == DTSDF_SDF_F32 && p.w_fmt == DTSDF_W_F32) return 0;
  if (p.sdf_fmt == DTSDF_SDF_F16 && p.w_fmt == DTSDF_W_U8) return 1;
  if (p.sdf_fmt == DTSDF_SDF_I16 && p.w_fmt == DTSDF_W_U8) return 2;
  return -1;
}

struct MapView {
  const HashEntry* entries;
  uint32_t mask;            // buckets - 1
  int fmt;
  void* geo;
  uint32_t* rgb;
  float* wc;
  const int4* bkey;
  uint32_t capacity;
  const GridRec* grid_rec;
  const uint64_t* grid_cell;
  const uint8_t* grid_group;
  int gx0, gy0, gz0;        // grid origin (block coordinates)
  int gx, gy, gz;           // grid dimensions (blocks)
  double voxel, inv_voxel;
  float tau, theta, w_carve, w_max, w_min;
  double step;
  int with_color;
};

// Slot of a block key, -1 if absent.  At most `mask + 1` probes.
__device__ inline int find_slot(const HashEntry* __restrict__ e, uint32_t mask, uint64_t key) {
  uint32_t s = hash_key(key) & mask;
  for (uint32_t i = 0; i <= mask; ++i) {
    uint64_t k = e[s].key;
    if (k == key) return (int)s;
    if (k == kEmptyKey) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

__device__ inline double floor_d(double x) { return floor(x); }

// Direction membership weight of Sec. 3 (eq. direction_weight), read as the clamped-linear
// function that is 1 for angles up to pi/2 - theta, 0 from theta on and linear in between.
// `c` is the cosine <n, v^D>.
__device__ inline float w_dir_cos(float c, float theta) {
  c = fminf(1.0f, fmaxf(-1.0f, c));
  float a = acosf(c);
  float v = (theta - a) / (2.0f * theta - 1.5707963267948966f);
  return fminf(1.0f, fmaxf(0.0f, v));
}

// <n, v^D> for direction D (X+, X-, Y+, Y-, Z+, Z-).
__device__ __host__ inline float axis_dot(float nx, float ny, float nz, int d) {
  float c = (d < 2) ? nx : (d < 4 ? ny : nz);
  return (d & 1) ? -c : c;
}

// Inserts (key, D) into the hash: the key by CAS on an empty slot, D as a request bit.
// New keys are refused (and counted as dropped requests) once `max_entries` slots are
// occupied, so that probe sequences of absent keys stay short.
__device__ inline void insert_request(HashEntry* e, uint32_t* req, uint32_t mask, uint64_t key, int d,
                               int32_t* counters, int32_t max_entries) {
  uint32_t s = hash_key(key) & mask;
  for (uint32_t i = 0; i <= mask; ++i) {
    unsigned long long* kp = reinterpret_cast<unsigned long long*>(&e[s].key);
    uint64_t k = __atomic_load_n(kp, __ATOMIC_RELAXED);
    if (k == kEmptyKey) {
      if (__atomic_load_n(&counters[3], __ATOMIC_RELAXED) >= max_entries) {
        atomicAdd(&counters[1], 1);
        return;
      }
      uint64_t prev = atomicCAS(kp, (unsigned long long)kEmptyKey, (unsigned long long)key);
      if (prev == kEmptyKey) atomicAdd(&counters[3], 1);
      if (prev == kEmptyKey || prev == key) {
        atomicOr(&req[s], 1u << d);
        return;
      }
      k = prev;
    }
    if (k == key) {
      atomicOr(&req[s], 1u << d);
      return;
    }
    s = (s + 1) & mask;
  }
  atomicExch(&counters[2], 1);
}

#define DTSDF_HIP(x)                                  \
  do {                                                \
    hipError_t e__ = (x);                             \
    if (e__ != hipSuccess) return DTSDF_E_HIP;        \
  } while (0)

}  // namespace dtsdf

// Host-side state of a map.
struct dtsdf_map {
  dtsdf_params p;
  int device;
  uint32_t buckets;
  dtsdf::HashEntry* entries;
  uint32_t* req;
  int4* bkey;
  void* geo;
  uint32_t* rgb;
  float* wc;
  int fmt;              // storage format (see Vox)
  int32_t* counters;
  int64_t n_bricks;     // host mirror of the bricks in use
  int64_t n_blocks;     // host mirror of occupied entries (updated on sync points)
  int64_t dropped;
  float* sub_min;
  float* slot_min;
  uint64_t* brick_neg;
  uint64_t* block_neg;
  dtsdf::GridRec* grid_rec;
  uint64_t* grid_cell;
  uint8_t* grid_group;
  uint8_t* mip;         // occupancy levels 1..kMipLevels, level l at mip_off[l]
  int64_t mip_off[dtsdf::kMipLevels + 2];
  int32_t grid_lo[3], grid_dim[3];
  int64_t grid_cap;     // allocated grid cells
  int64_t mip_cap;      // allocated mip bytes
  // 1: a regular (single-volume) TSDF written by dtsdf_combine: direction slot 0 holds the
  // combined value with weight 1 (0: no value), rendered without direction weighting
  int regular;
  int64_t mirrored;     // source block count at the last block mirroring (-1: never)
  // recycled bricks (Sec. 3): pool indices freed by dtsdf_recycle, taken before the pool
  // grows; counters[10] holds their number on the device, n_free its host mirror
  int32_t* free_list;
  int64_t n_free;
  // deterministic allocation: the frame's new (block key << 3 | D) requests and their hash
  // slots, double buffered for the radix sort, and the sort's scratch (grown on demand)
  uint64_t* alloc_keys;
  uint32_t* alloc_vals;
  int64_t alloc_cap;
  void* sort_tmp;
  size_t sort_tmp_bytes;
  // bricks whose voxels may project into the frame being fused (counters[11] of them)
  int32_t* vis_list;
  // per listed brick of the frame: voxels whose distance / colour were updated (allocated
  // on the first integration that asks for statistics)
  int2* fuse_cnt;
  // per pixel of the frame being fused: 1 if no valid depth within two pixels differs from
  // the pixel's by more than tau (the carving guard of Sec. 3)
  uint8_t* carve_ok;
  int64_t carve_cap;
  // integration scratch, grown on demand
  int64_t img_cap;
  float* vmap;
  float* nmap;
};

namespace dtsdf {
MapView make_view(const dtsdf_map* m);

// Slot of the per-device descriptor staging ring (staging.hip): pinned host memory, device
// memory and an event recorded behind the last work that read the slot.
struct Stage {
  uint8_t* host = nullptr;
  uint8_t* dev = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  bool recorded = false;
};
constexpr size_t kStageHostBytes = size_t(2) << 20;
constexpr size_t kStageDevBytes = size_t(8) << 20;
// Hands out a free slot of the current device once the work that last used it has
// finished (DTSDF_E_BUSY if every slot is held by a call that has not released it).
dtsdf_status stage_acquire(Stage** out);
// Records the slot's event on `st` behind the work enqueued so far and frees the slot.
dtsdf_status stage_release(Stage* s, hipStream_t st);
// Enqueues the clamp of the bricks-handed-out counter (counters[0]) at the pool capacity.
void launch_clamp_handed(dtsdf_map* m, hipStream_t st);

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Minima of the eight 4^3 sub-blocks of brick `b` over voxels with w > 0 (+inf if none),
// written to out8[0..7], the brick's non-positive voxel mask (w > 0, sdf <= kSkipMin;
// word z, bit x + 8 y) written to bits16[0..7] and its observed voxel mask (w > 0) to
// bits16[8..15]; called by every thread of a 256-thread workgroup.
template <int F>
__device__ inline void brick_sub_min(const void* geo, size_t b, float* out8, uint64_t* bits16) {
  __shared__ float vals[kVox];
  for (int l = threadIdx.x; l < kVox; l += blockDim.x) {
    float sd, w;
    Vox<F>::load(geo, b * kVox + l, sd, w);
    vals[l] = w > 0.f ? sd : INFINITY;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < 2; ++q) {
    const int sb = 2 * wave + q;
    const int lx = (lane & 3) + 4 * (sb & 1), ly = ((lane >> 2) & 3) + 4 * ((sb >> 1) & 1),
              lz = (lane >> 4) + 4 * (sb >> 2);
    float v = vals[lx + 8 * ly + 64 * lz];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    if (lane == 0) out8[sb] = v;
    const int z = 2 * wave + q;
    const float vz = vals[lane + 64 * z];
    const uint64_t neg = __ballot(vz <= kSkipMin);
    const uint64_t obs = __ballot(vz < INFINITY);
    if (lane == 0) {
      bits16[z] = neg;
      bits16[8 + z] = obs;
    }
  }
  __syncthreads();
}
// Recomputes sub_min and brick_neg of every brick in use.
dtsdf_status brick_stats(dtsdf_map* m, hipStream_t st);
// Enqueues the bounding-box reduction into counters[4..9].
void launch_bbox(dtsdf_map* m, hipStream_t st);
// Makes the grid cover the bounding box `hb` (host copy); reallocates and clears on growth.
dtsdf_status ensure_grid(dtsdf_map* m, const int32_t* hb, hipStream_t st);
// Enqueues the slot scatter and the skip codes.
dtsdf_status launch_index_update(dtsdf_map* m, hipStream_t st);
// All of the above (synchronises `st`).
dtsdf_status rebuild_index(dtsdf_map* m, hipStream_t st);
// Pool indices for the requested (block, D) bricks without one, handed out in ascending
// (block key, D) order (recycled indices first, in ascending order, then the pool's unused
// end), so the pool layout and the requests dropped at capacity do not depend on thread
// order.  Synchronises `st` once (the request count sizes the sort).
dtsdf_status launch_assign(dtsdf_map* m, hipStream_t st);
// Sorts the free list ascending (after recycling pushed to it in thread order).
dtsdf_status sort_free_list(dtsdf_map* m, hipStream_t st);
// rebuild_index with every grid cell cleared first (blocks may have disappeared).
dtsdf_status rebuild_index_cleared(dtsdf_map* m, hipStream_t st);
}
