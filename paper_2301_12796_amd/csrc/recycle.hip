// Recycling of bricks that hold no surface (Sec. 3: blocks allocated by stray points that
// repeated carving has turned into free space are returned to the pool).
//
// A brick is recycled when every observed voxel (w > 0) of it holds a value of at least
// t_free (in units of the truncation distance; carving drives values towards 1), or when it
// has no observed voxel at all.  The test reads the per-brick sub-block minima that fusion
// keeps up to date, so a pass costs one read of eight floats per brick in use.
//
//   recycle_k      one thread per hash slot: frees the qualifying directions of the slot's
//                  block, pushes their pool indices onto the free list and marks them
//   clear_freed_k  one workgroup per pool brick: a brick freed by this pass is reset to the
//                  state of an unused pool brick (zero distance, weight, colour; empty
//                  summaries) and its direction set to -1
// The render index is then rebuilt from a cleared grid, since blocks may have vanished.
#include <cmath>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

constexpr int kFreedNow = -2;

__global__ __launch_bounds__(256) void recycle_k(HashEntry* entries, uint32_t buckets,
                                                 const float* __restrict__ sub_min, int4* bkey,
                                                 int32_t* free_list, int32_t* counters,
                                                 float t_free) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= buckets) return;
  if (entries[s].key == kEmptyKey) return;
  for (int d = 0; d < 6; ++d) {
    const int32_t b = entries[s].brick[d];
    if (b < 0) continue;
    float mn = sub_min[(size_t)b * 8];
    for (int k = 1; k < 8; ++k) mn = fminf(mn, sub_min[(size_t)b * 8 + k]);
    if (!(mn >= t_free)) continue;
    entries[s].brick[d] = -1;
    const int f = atomicAdd(&counters[10], 1);
    free_list[f] = b;
    bkey[b].w = kFreedNow;
  }
}

__global__ __launch_bounds__(256) void clear_freed_k(int4* bkey, uint32_t* geo_words,
                                                     int words_per_brick, uint32_t* rgb,
                                                     float* wc, float* sub_min,
                                                     uint64_t* brick_neg) {
  const size_t b = blockIdx.x;
  const bool freed = bkey[b].w == kFreedNow;
  __syncthreads();
  if (!freed) return;
  for (int i = threadIdx.x; i < words_per_brick; i += blockDim.x)
    geo_words[b * words_per_brick + i] = 0u;
  for (int i = threadIdx.x; i < kVox; i += blockDim.x) {
    if (rgb) rgb[b * kVox + i] = 0u;
    if (wc) wc[b * kVox + i] = 0.f;
  }
  if (threadIdx.x < 8) sub_min[b * 8 + threadIdx.x] = __int_as_float(0x7f7f7f7f);
  if (threadIdx.x < 16) brick_neg[b * 16 + threadIdx.x] = 0ull;
  if (threadIdx.x == 0) bkey[b].w = -1;
}

}  // namespace

extern "C" dtsdf_status dtsdf_recycle(dtsdf_map* m, float t_free, int64_t* recycled,
                                      void* stream) {
  if (!m || m->regular || m->p.dense || !(t_free > 0.f) || !std::isfinite(t_free))
    return DTSDF_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!m->free_list) {
    DTSDF_HIP(hipStreamSynchronize(st));
    if (hipMalloc(&m->free_list, sizeof(int32_t) * m->p.brick_capacity) != hipSuccess) {
      m->free_list = nullptr;
      return DTSDF_E_NOMEM;
    }
  }
  const int64_t before = m->n_free;
  hipLaunchKernelGGL(recycle_k, dim3((m->buckets + 255) / 256), dim3(256), 0, st, m->entries,
                     m->buckets, m->sub_min, m->bkey, m->free_list, m->counters, t_free);
  if (m->n_bricks > 0) {
    const int gb = m->fmt == 0 ? (int)Vox<0>::kGeoBytes : (int)VoxPacked::kGeoBytes;
    const int words = kVox * gb / 4;
    hipLaunchKernelGGL(clear_freed_k, dim3((uint32_t)m->n_bricks), dim3(256), 0, st, m->bkey,
                       reinterpret_cast<uint32_t*>(m->geo), words, m->rgb, m->wc, m->sub_min,
                       m->brick_neg);
  }
  DTSDF_HIP(hipGetLastError());
  int32_t nf = 0;
  DTSDF_HIP(hipMemcpyAsync(&nf, m->counters + 10, sizeof(nf), hipMemcpyDeviceToHost, st));
  DTSDF_HIP(hipStreamSynchronize(st));
  m->n_free = nf;
  if (recycled) *recycled = nf - before;
  // the free list was pushed in thread order: sorted, allocation hands its indices out in a
  // fixed order
  const dtsdf_status ss = sort_free_list(m, st);
  if (ss != DTSDF_OK) return ss;
  return rebuild_index_cleared(m, st);
}
