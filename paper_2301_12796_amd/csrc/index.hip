// Per-brick summaries and the dense render index (see dtsdf_internal.hpp).
#include <algorithm>
#include <climits>
#include <cmath>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

// Sub-block minima of every brick in use; one workgroup per brick.
template <int F>
__global__ __launch_bounds__(256) void brick_stats_k(const void* geo, float* sub_min,
                                                     uint64_t* brick_neg) {
  brick_sub_min<F>(geo, blockIdx.x, sub_min + (size_t)blockIdx.x * 8,
                   brick_neg + (size_t)blockIdx.x * 16);
}

__device__ inline bool slot_present(const HashEntry& e) {
  if (e.key == kEmptyKey) return false;
  for (int d = 0; d < 6; ++d)
    if (e.brick[d] >= 0) return true;
  return false;
}

// Bounding box of the occupied blocks: min/max folded across the wave with xor shuffles and
// across the workgroup in LDS, so each workgroup issues six atomics.
// A fixed grid strides over the table, so that few workgroups contend for the six atomics.
constexpr int kBboxBlocks = 512;
__global__ __launch_bounds__(256) void bbox_k(const HashEntry* __restrict__ e, uint32_t buckets,
                                              int32_t* bbox) {
  int v[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < buckets;
       s += gridDim.x * blockDim.x) {
    const HashEntry ent = e[s];
    if (slot_present(ent)) {
      int b[3];
      unpack_key(ent.key, b[0], b[1], b[2]);
      for (int k = 0; k < 3; ++k) {
        v[k] = min(v[k], b[k]);
        v[3 + k] = max(v[3 + k], b[k]);
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[k] = min(v[k], __shfl_xor(v[k], off, 64));
      v[3 + k] = max(v[3 + k], __shfl_xor(v[3 + k], off, 64));
    }
  __shared__ int part[4][6];
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) part[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    int r = part[0][k];
    for (int w = 1; w < 4; ++w) r = k < 3 ? min(r, part[w][k]) : max(r, part[w][k]);
    if (k < 3 && r != INT_MAX) atomicMin(&bbox[k], r);
    if (k >= 3 && r != INT_MIN) atomicMax(&bbox[k], r);
  }
}

__global__ __launch_bounds__(256) void grid_clear_k(GridRec* rec, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  GridRec r;
  for (int d = 0; d < 6; ++d) r.brick[d] = -1;
  r.info = 0;
  r.slot = -1;
  rec[i] = r;
}

__global__ __launch_bounds__(256) void bytes_clear_k(uint8_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

struct Grid {
  int x0, y0, z0, nx, ny, nz;
  int64_t mip_off[kMipLevels + 2];   // byte offset of occupancy level l (1 .. kMipLevels)
  __device__ int64_t index(int bx, int by, int bz) const {
    int ix = bx - x0, iy = by - y0, iz = bz - z0;
    if (ix < 0 || iy < 0 || iz < 0 || ix >= nx || iy >= ny || iz >= nz) return -1;
    return ((int64_t)iz * ny + iy) * nx + ix;
  }
  // cell of occupancy level l holding grid block (ix, iy, iz)
  __device__ int64_t mip_index(int l, int ix, int iy, int iz) const {
    const int mx = (nx + (1 << l) - 1) >> l, my = (ny + (1 << l) - 1) >> l;
    return mip_off[l] + ((int64_t)(iz >> l) * my + (iy >> l)) * mx + (ix >> l);
  }
};

// Records of the present blocks (bricks and hash slot) and their occupancy at every level.
__global__ __launch_bounds__(256) void grid_scatter_k(const HashEntry* __restrict__ e,
                                                      uint32_t buckets, Grid g, GridRec* rec,
                                                      uint8_t* mip) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  int b[3];
  unpack_key(ent.key, b[0], b[1], b[2]);
  int64_t i = g.index(b[0], b[1], b[2]);
  if (i < 0) return;
  for (int d = 0; d < 6; ++d) rec[i].brick[d] = ent.brick[d];
  rec[i].slot = (int32_t)s;
  const int ix = b[0] - g.x0, iy = b[1] - g.y0, iz = b[2] - g.z0;
  for (int l = 1; l <= kMipLevels; ++l) mip[g.mip_index(l, ix, iy, iz)] = 1;
}

// Empty level of every absent block: the largest l <= kMipLevels whose aligned cell of 2^l
// blocks per edge holds no present block (0: only the block itself is known empty).
__global__ __launch_bounds__(256) void empty_level_k(Grid g, GridRec* rec,
                                                     const uint8_t* __restrict__ mip) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.nx * g.ny * g.nz) return;
  if (rec[i].slot >= 0) return;
  const int ix = (int)(i % g.nx), iy = (int)((i / g.nx) % g.ny), iz = (int)(i / ((int64_t)g.nx * g.ny));
  uint32_t e = 0;
  for (int l = 1; l <= kMipLevels; ++l) {
    if (mip[g.mip_index(l, ix, iy, iz)]) break;
    e = (uint32_t)l;
  }
  rec[i].info = e << 8;
}

// Per entry and sub-block: min over the block's directions of the sub-block minima.
__global__ __launch_bounds__(256) void slot_min_k(const HashEntry* __restrict__ e,
                                                  uint32_t buckets,
                                                  const float* __restrict__ sub_min,
                                                  float* slot_min) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  float mn[8];
  for (int q = 0; q < 8; ++q) mn[q] = INFINITY;
  for (int d = 0; d < 6; ++d) {
    const int br = ent.brick[d];
    if (br < 0) continue;
    for (int q = 0; q < 8; ++q) mn[q] = fminf(mn[q], sub_min[(size_t)br * 8 + q]);
  }
  for (int q = 0; q < 8; ++q) slot_min[(size_t)s * 8 + q] = mn[q];
}

// Skip mask of every present block: bit q is set if the minima of the 2x2x2 sub-blocks
// starting at sub-block q (possibly in the +x/+y/+z neighbour blocks) all exceed kSkipMin;
// those sub-blocks hold every corner a cell based in sub-block q can reach.  Absent
// neighbours make the cells that need them undefined and do not constrain the mask.
__global__ __launch_bounds__(256) void grid_mask_k(const HashEntry* __restrict__ e,
                                                   uint32_t buckets, Grid g, GridRec* rec,
                                                   const float* __restrict__ slot_min) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  int b[3];
  unpack_key(ent.key, b[0], b[1], b[2]);
  int64_t i = g.index(b[0], b[1], b[2]);
  if (i < 0) return;
  int nslot[8];
  for (int o = 0; o < 8; ++o) {
    int64_t j = o == 0 ? i : g.index(b[0] + (o & 1), b[1] + ((o >> 1) & 1), b[2] + ((o >> 2) & 1));
    nslot[o] = o == 0 ? (int)s : (j < 0 ? -1 : rec[j].slot);
  }
  uint32_t bits = 0;
  for (int q = 0; q < 8; ++q) {
    const int qs[3] = {q & 1, (q >> 1) & 1, q >> 2};
    float mn = INFINITY;
    for (int dd = 0; dd < 8; ++dd) {
      const int t[3] = {qs[0] + (dd & 1), qs[1] + ((dd >> 1) & 1), qs[2] + (dd >> 2)};
      const int o = (t[0] >> 1) | ((t[1] >> 1) << 1) | ((t[2] >> 1) << 2);
      const int sub = (t[0] & 1) | ((t[1] & 1) << 1) | ((t[2] & 1) << 2);
      const int sl = nslot[o];
      if (sl >= 0) mn = fminf(mn, slot_min[(size_t)sl * 8 + sub]);
    }
    if (mn > kSkipMin) bits |= 1u << q;
  }
  rec[i].info = bits | kRecPresent;
}

// Per entry and slice z: OR of the non-positive voxel masks of the block's bricks.
__global__ __launch_bounds__(256) void block_neg_k(const HashEntry* __restrict__ e,
                                                   uint32_t buckets,
                                                   const uint64_t* __restrict__ brick_neg,
                                                   uint64_t* block_neg) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t s = (uint32_t)(t >> 3);
  const int z = (int)(t & 7);
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  uint64_t v = 0;
  for (int d = 0; d < 6; ++d)
    if (ent.brick[d] >= 0) v |= brick_neg[(size_t)ent.brick[d] * 16 + z];
  block_neg[(size_t)s * 8 + z] = v;
}

// OR of a voxel slice over x and x + 1 (x + 1 of the last column from the +x neighbour's
// slice `nx`).
__device__ inline uint64_t or_x(uint64_t w, uint64_t nx) {
  constexpr uint64_t kCol0 = 0x0101010101010101ull, kCol7 = 0x8080808080808080ull;
  return w | ((w >> 1) & ~kCol7) | ((nx & kCol0) << 7);
}

// OR over (x, x + 1) x (y, y + 1) of a slice, given the slices of the +x, +y and +xy blocks.
__device__ inline uint64_t or_xy(uint64_t w, uint64_t nx, uint64_t ny, uint64_t nxy) {
  const uint64_t r = or_x(w, nx), ry = or_x(ny, nxy);
  return r | (r >> 8) | ((ry & 0xFFull) << 56);
}

// Positive-cell mask of every present block (see cell_mask in dtsdf_internal.hpp): a cell is
// positive if none of its corners is non-positive in any direction of the block holding it.
// Absent neighbours hold no values: cells that would need them are undefined in every
// direction that lacks a corner, so they do not constrain the mask.
__global__ __launch_bounds__(256) void cell_mask_k(const HashEntry* __restrict__ e,
                                                   uint32_t buckets, Grid g,
                                                   const GridRec* __restrict__ rec,
                                                   const uint64_t* __restrict__ block_neg,
                                                   uint64_t* grid_cell) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t s = (uint32_t)(t >> 3);
  const int z = (int)(t & 7);
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  int b[3];
  unpack_key(ent.key, b[0], b[1], b[2]);
  const int64_t i = g.index(b[0], b[1], b[2]);
  if (i < 0) return;
  // slices z and z + 1 of the blocks at offsets 0, +x, +y, +xy (z + 1 = 8: slice 0 of the
  // blocks one further in z)
  uint64_t w[2][4];
  for (int h = 0; h < 2; ++h) {
    const int zz = z + h;
    const int oz = zz >> 3;
    for (int q = 0; q < 4; ++q) {
      const int ox = q & 1, oy = q >> 1;
      int sl = -1;
      if (ox == 0 && oy == 0 && oz == 0) {
        sl = (int)s;
      } else {
        const int64_t j = g.index(b[0] + ox, b[1] + oy, b[2] + oz);
        sl = j < 0 ? -1 : rec[j].slot;
      }
      w[h][q] = sl < 0 ? 0ull : block_neg[(size_t)sl * 8 + (zz & 7)];
    }
  }
  const uint64_t neg = or_xy(w[0][0], w[0][1], w[0][2], w[0][3]) |
                       or_xy(w[1][0], w[1][1], w[1][2], w[1][3]);
  grid_cell[(size_t)i * 8 + z] = ~neg;
}

// AND of a voxel slice over x and x + 1, and over (x, x + 1) x (y, y + 1) (see or_x).
__device__ inline uint64_t and_x(uint64_t w, uint64_t nx) {
  constexpr uint64_t kCol0 = 0x0101010101010101ull, kCol7 = 0x8080808080808080ull;
  return w & (((w >> 1) & ~kCol7) | ((nx & kCol0) << 7));
}

__device__ inline uint64_t and_xy(uint64_t w, uint64_t nx, uint64_t ny, uint64_t nxy) {
  const uint64_t r = and_x(w, nx), ry = and_x(ny, nxy);
  return r & ((r >> 8) | ((ry & 0xFFull) << 56));
}

// Defined-direction bytes of every present block (see dir_groups in dtsdf_internal.hpp):
// one thread per block and slab of cells z = 2 gz, 2 gz + 1, writing the 16 group bytes of
// that slab.  A cell is defined in D if its 8 corners (in the +x/+y/+z neighbours where it
// leaves the block) are observed in D.
__global__ __launch_bounds__(256) void dir_groups_k(const HashEntry* __restrict__ e,
                                                    uint32_t buckets, Grid g,
                                                    const GridRec* __restrict__ rec,
                                                    const uint64_t* __restrict__ brick_bits,
                                                    uint8_t* grid_group) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t s = (uint32_t)(t >> 2);
  const int gz = (int)(t & 3);
  if (s >= buckets) return;
  const HashEntry ent = e[s];
  if (!slot_present(ent)) return;
  int b[3];
  unpack_key(ent.key, b[0], b[1], b[2]);
  const int64_t i = g.index(b[0], b[1], b[2]);
  if (i < 0) return;
  // grid records of the blocks at offsets (ox, oy, oz), index ox + 2 oy + 4 oz (-1: outside)
  int64_t nb[8];
  nb[0] = i;
  for (int o = 1; o < 8; ++o)
    nb[o] = g.index(b[0] + (o & 1), b[1] + ((o >> 1) & 1), b[2] + ((o >> 2) & 1));
  uint32_t bytes[4] = {0u, 0u, 0u, 0u};   // 16 group bytes of the slab
  for (int d = 0; d < 6; ++d) {
    if (ent.brick[d] < 0) continue;
    int br[8];
    br[0] = ent.brick[d];
    for (int o = 1; o < 8; ++o) br[o] = nb[o] < 0 ? -1 : rec[nb[o]].brick[d];
    // observed words of slices 2 gz .. 2 gz + 2 for the blocks at (0,0), (+x), (+y), (+xy)
    uint64_t w[3][4];
    for (int h = 0; h < 3; ++h) {
      const int zz = 2 * gz + h;
      const int oz = zz >> 3;
      for (int q = 0; q < 4; ++q) {
        const int bb = br[q + 4 * oz];
        w[h][q] = bb < 0 ? 0ull : brick_bits[(size_t)bb * 16 + 8 + (zz & 7)];
      }
    }
    const uint64_t c0 = and_xy(w[0][0], w[0][1], w[0][2], w[0][3]) &
                        and_xy(w[1][0], w[1][1], w[1][2], w[1][3]);
    const uint64_t c1 = and_xy(w[1][0], w[1][1], w[1][2], w[1][3]) &
                        and_xy(w[2][0], w[2][1], w[2][2], w[2][3]);
    const uint64_t u = c0 | c1;
    for (int gy = 0; gy < 4; ++gy)
      for (int gx = 0; gx < 4; ++gx)
        if ((u >> (2 * gx + 16 * gy)) & 0x0303ull)
          bytes[gy] |= (1u << d) << (8 * gx);
  }
  uint32_t* out = reinterpret_cast<uint32_t*>(grid_group + (size_t)i * 64 + 16 * gz);
  for (int gy = 0; gy < 4; ++gy) out[gy] = bytes[gy];
}

// Also clamps the free-list count (counters[10]) at zero (pops by the allocation that ran
// before may have driven it below) and clears the visible-brick count (counters[11]).
__global__ void bbox_reset_k(int32_t* counters) {
  if (threadIdx.x < 3) counters[4 + threadIdx.x] = INT_MAX;
  else if (threadIdx.x < 6) counters[4 + threadIdx.x] = INT_MIN;
  else if (threadIdx.x == 6 && counters[10] < 0) counters[10] = 0;
  else if (threadIdx.x == 7) counters[11] = 0;
}

}  // namespace

namespace dtsdf {

dtsdf_status brick_stats(dtsdf_map* m, hipStream_t st) {
  if (m->n_bricks > 0) {
    const dim3 g((uint32_t)m->n_bricks);
    if (m->fmt == 0)
      hipLaunchKernelGGL(brick_stats_k<0>, g, dim3(256), 0, st, m->geo, m->sub_min, m->brick_neg);
    else if (m->fmt == 1)
      hipLaunchKernelGGL(brick_stats_k<1>, g, dim3(256), 0, st, m->geo, m->sub_min, m->brick_neg);
    else
      hipLaunchKernelGGL(brick_stats_k<2>, g, dim3(256), 0, st, m->geo, m->sub_min, m->brick_neg);
  }
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

void launch_bbox(dtsdf_map* m, hipStream_t st) {
  int32_t* bbox = m->counters + 4;
  hipLaunchKernelGGL(bbox_reset_k, dim3(1), dim3(64), 0, st, m->counters);
  const uint32_t blocks = std::min<uint32_t>((m->buckets + 255) / 256, kBboxBlocks);
  hipLaunchKernelGGL(bbox_k, dim3(blocks), dim3(256), 0, st, m->entries, m->buckets, bbox);
}

namespace {

Grid grid_of(const dtsdf_map* m) {
  Grid g{m->grid_lo[0], m->grid_lo[1], m->grid_lo[2], m->grid_dim[0], m->grid_dim[1],
         m->grid_dim[2], {}};
  for (int l = 0; l < kMipLevels + 2; ++l) g.mip_off[l] = m->mip_off[l];
  return g;
}

// Byte offsets of the occupancy levels 1 .. kMipLevels for a grid of `dim` blocks; returns
// the total size.
int64_t mip_layout(const int dim[3], int64_t off[kMipLevels + 2]) {
  int64_t total = 0;
  off[0] = 0;
  for (int l = 1; l <= kMipLevels; ++l) {
    off[l] = total;
    total += (int64_t)ceil_div(dim[0], 1 << l) * ceil_div(dim[1], 1 << l) * ceil_div(dim[2], 1 << l);
  }
  off[kMipLevels + 1] = total;
  return total;
}

// Clears every record and the occupancy levels of the current grid.
dtsdf_status clear_grid(dtsdf_map* m, hipStream_t st) {
  const int64_t cells = (int64_t)m->grid_dim[0] * m->grid_dim[1] * m->grid_dim[2];
  const int64_t mb = m->mip_off[kMipLevels + 1];
  hipLaunchKernelGGL(grid_clear_k, dim3((uint32_t)((cells + 255) / 256)), dim3(256), 0, st,
                     m->grid_rec, cells);
  hipLaunchKernelGGL(bytes_clear_k, dim3((uint32_t)((mb + 255) / 256)), dim3(256), 0, st,
                     m->mip, mb);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

}  // namespace

dtsdf_status ensure_grid(dtsdf_map* m, const int32_t* hb, hipStream_t st) {
  const bool empty = hb[0] > hb[3];
  if (empty) {
    for (int k = 0; k < 3; ++k) m->grid_dim[k] = 0;
    return DTSDF_OK;
  }
  bool inside = m->grid_dim[0] > 0;
  for (int k = 0; k < 3 && inside; ++k)
    inside = hb[k] >= m->grid_lo[k] && hb[3 + k] < m->grid_lo[k] + m->grid_dim[k];
  if (inside) return DTSDF_OK;
  // new grid: bounding box padded by 8 blocks per side so that growth is rare
  const int pad = m->p.dense ? 1 : 8;
  int lo[3], dim[3];
  int64_t cells = 1;
  for (int k = 0; k < 3; ++k) {
    lo[k] = hb[k] - pad;
    dim[k] = hb[3 + k] - hb[k] + 1 + 2 * pad;
    cells *= dim[k];
  }
  if (cells > kMaxGridBlocks) return DTSDF_E_CAPACITY;
  int64_t off[kMipLevels + 2];
  const int64_t mb = mip_layout(dim, off);
  if (cells > m->grid_cap || mb > m->mip_cap) {
    DTSDF_HIP(hipStreamSynchronize(st));
    (void)hipFree(m->grid_rec);
    (void)hipFree(m->grid_cell);
    (void)hipFree(m->grid_group);
    (void)hipFree(m->mip);
    m->grid_rec = nullptr;
    m->grid_cell = nullptr;
    m->grid_group = nullptr;
    m->mip = nullptr;
    m->grid_cap = 0;
    m->mip_cap = 0;
    for (int k = 0; k < 3; ++k) m->grid_dim[k] = 0;
    const int64_t want = cells + cells / 4;
    const int64_t wantm = mb + mb / 4 + 64;
    if (hipMalloc(&m->grid_rec, sizeof(GridRec) * want) != hipSuccess ||
        hipMalloc(&m->grid_cell, sizeof(uint64_t) * 8 * want) != hipSuccess ||
        hipMalloc(&m->grid_group, (size_t)64 * want) != hipSuccess ||
        hipMalloc(&m->mip, wantm) != hipSuccess)
      return DTSDF_E_NOMEM;
    m->grid_cap = want;
    m->mip_cap = wantm;
  }
  for (int k = 0; k < 3; ++k) {
    m->grid_lo[k] = lo[k];
    m->grid_dim[k] = dim[k];
  }
  for (int l = 0; l < kMipLevels + 2; ++l) m->mip_off[l] = off[l];
  return clear_grid(m, st);
}

dtsdf_status launch_index_update(dtsdf_map* m, hipStream_t st) {
  if (m->grid_dim[0] == 0) return DTSDF_OK;
  const Grid g = grid_of(m);
  const int64_t cells = (int64_t)m->grid_dim[0] * m->grid_dim[1] * m->grid_dim[2];
  const dim3 grd((m->buckets + 255) / 256);
  hipLaunchKernelGGL(grid_scatter_k, grd, dim3(256), 0, st, m->entries, m->buckets, g,
                     m->grid_rec, m->mip);
  hipLaunchKernelGGL(empty_level_k, dim3((uint32_t)((cells + 255) / 256)), dim3(256), 0, st, g,
                     m->grid_rec, m->mip);
  hipLaunchKernelGGL(slot_min_k, grd, dim3(256), 0, st, m->entries, m->buckets, m->sub_min,
                     m->slot_min);
  hipLaunchKernelGGL(grid_mask_k, grd, dim3(256), 0, st, m->entries, m->buckets, g,
                     m->grid_rec, m->slot_min);
  const dim3 grd8((uint32_t)(((uint64_t)m->buckets * 8 + 255) / 256));
  hipLaunchKernelGGL(block_neg_k, grd8, dim3(256), 0, st, m->entries, m->buckets, m->brick_neg,
                     m->block_neg);
  hipLaunchKernelGGL(cell_mask_k, grd8, dim3(256), 0, st, m->entries, m->buckets, g,
                     m->grid_rec, m->block_neg, m->grid_cell);
  const dim3 grd4((uint32_t)(((uint64_t)m->buckets * 4 + 255) / 256));
  hipLaunchKernelGGL(dir_groups_k, grd4, dim3(256), 0, st, m->entries, m->buckets, g,
                     m->grid_rec, m->brick_neg, m->grid_group);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

dtsdf_status rebuild_index(dtsdf_map* m, hipStream_t st) {
  launch_bbox(m, st);
  int32_t hb[6];
  DTSDF_HIP(hipMemcpyAsync(hb, m->counters + 4, sizeof(hb), hipMemcpyDeviceToHost, st));
  DTSDF_HIP(hipStreamSynchronize(st));
  dtsdf_status s = ensure_grid(m, hb, st);
  if (s != DTSDF_OK) return s;
  return launch_index_update(m, st);
}

dtsdf_status rebuild_index_cleared(dtsdf_map* m, hipStream_t st) {
  launch_bbox(m, st);
  int32_t hb[6];
  DTSDF_HIP(hipMemcpyAsync(hb, m->counters + 4, sizeof(hb), hipMemcpyDeviceToHost, st));
  DTSDF_HIP(hipStreamSynchronize(st));
  dtsdf_status s = ensure_grid(m, hb, st);
  if (s != DTSDF_OK) return s;
  if (m->grid_dim[0] == 0) return DTSDF_OK;
  s = clear_grid(m, st);
  if (s != DTSDF_OK) return s;
  return launch_index_update(m, st);
}

}  // namespace dtsdf
