// Map lifetime, parameter validation, import/export of the voxel-block pool.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace dtsdf {

MapView make_view(const dtsdf_map* m) {
  MapView v;
  v.entries = m->entries;
  v.mask = m->buckets - 1;
  v.fmt = m->fmt;
  v.geo = m->geo;
  v.rgb = m->rgb;
  v.wc = m->wc;
  v.bkey = m->bkey;
  v.capacity = m->p.brick_capacity;
  v.grid_rec = m->grid_rec;
  v.grid_cell = m->grid_cell;
  v.grid_group = m->grid_group;
  v.gx0 = m->grid_lo[0];
  v.gy0 = m->grid_lo[1];
  v.gz0 = m->grid_lo[2];
  v.gx = m->grid_dim[0];
  v.gy = m->grid_dim[1];
  v.gz = m->grid_dim[2];
  v.voxel = (double)m->p.voxel_size;
  v.inv_voxel = 1.0 / (double)m->p.voxel_size;
  v.tau = m->p.truncation;
  v.theta = m->p.theta;
  v.w_carve = m->p.w_carve;
  v.w_max = m->p.w_max;
  v.w_min = m->p.w_min;
  v.step = (double)m->p.lattice_step;
  v.with_color = m->p.with_color;
  return v;
}

}  // namespace dtsdf

namespace {

struct HostKey {
  int32_t x, y, z, d;
};

bool key_less(const HostKey& a, const HostKey& b) {
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  if (a.z != b.z) return a.z < b.z;
  return a.d < b.d;
}

// Builds the hash table for a sorted brick list on the host: brick index = list position.
// Returns false if a key is out of range, duplicated, or the table overflows.
bool build_table(const std::vector<HostKey>& keys, uint32_t buckets,
                 std::vector<HashEntry>& entries, int64_t* n_blocks) {
  entries.assign(buckets, HashEntry{kEmptyKey, {-1, -1, -1, -1, -1, -1}});
  uint32_t mask = buckets - 1;
  int64_t blocks = 0;
  for (size_t i = 0; i < keys.size(); ++i) {
    const HostKey& k = keys[i];
    if (!key_in_range(k.x, k.y, k.z) || k.d < 0 || k.d > 5) return false;
    uint64_t pk = pack_key(k.x, k.y, k.z);
    uint32_t s = hash_key(pk) & mask;
    uint32_t probes = 0;
    while (entries[s].key != kEmptyKey && entries[s].key != pk) {
      s = (s + 1) & mask;
      if (++probes > mask) return false;
    }
    if (entries[s].key == kEmptyKey) {
      entries[s].key = pk;
      ++blocks;
    }
    if (entries[s].brick[k.d] >= 0) return false;   // duplicate key
    entries[s].brick[k.d] = (int32_t)i;
  }
  *n_blocks = blocks;
  return true;
}

dtsdf_status upload_table(dtsdf_map* m, const std::vector<HostKey>& keys) {
  std::vector<HashEntry> entries;
  int64_t blocks = 0;
  if (!build_table(keys, m->buckets, entries, &blocks)) return DTSDF_E_INVAL;
  std::vector<int4> bk(keys.size());
  for (size_t i = 0; i < keys.size(); ++i) bk[i] = make_int4(keys[i].x, keys[i].y, keys[i].z, keys[i].d);
  DTSDF_HIP(hipMemcpy(m->entries, entries.data(), sizeof(HashEntry) * m->buckets,
                      hipMemcpyHostToDevice));
  if (!bk.empty())
    DTSDF_HIP(hipMemcpy(m->bkey, bk.data(), sizeof(int4) * bk.size(), hipMemcpyHostToDevice));
  int32_t counters[16] = {(int32_t)keys.size(), 0, 0, (int32_t)blocks};
  DTSDF_HIP(hipMemcpy(m->counters, counters, sizeof(counters), hipMemcpyHostToDevice));
  m->n_bricks = (int64_t)keys.size();
  m->n_blocks = blocks;
  m->dropped = 0;
  m->n_free = 0;
  return DTSDF_OK;
}

void free_map(dtsdf_map* m) {
  if (!m) return;
  (void)hipFree(m->entries);
  (void)hipFree(m->req);
  (void)hipFree(m->bkey);
  (void)hipFree(m->geo);
  (void)hipFree(m->rgb);
  (void)hipFree(m->wc);
  (void)hipFree(m->counters);
  (void)hipFree(m->free_list);
  (void)hipFree(m->vis_list);
  (void)hipFree(m->fuse_cnt);
  (void)hipFree(m->alloc_keys);
  (void)hipFree(m->alloc_vals);
  (void)hipFree(m->sort_tmp);
  (void)hipFree(m->carve_ok);
  (void)hipFree(m->vmap);
  (void)hipFree(m->nmap);
  (void)hipFree(m->sub_min);
  (void)hipFree(m->slot_min);
  (void)hipFree(m->brick_neg);
  (void)hipFree(m->block_neg);
  (void)hipFree(m->grid_rec);
  (void)hipFree(m->grid_cell);
  (void)hipFree(m->grid_group);
  (void)hipFree(m->mip);
  delete m;
}

size_t geo_bytes(int fmt) { return fmt == 0 ? (size_t)Vox<0>::kGeoBytes : (size_t)VoxPacked::kGeoBytes; }

// Host encode / decode of one voxel in format F (same rounding as the device).
template <int F>
void host_store(void* geo, uint32_t* rgb, float* wc, size_t i, float s, float w,
                const uint8_t* c3, float cw, bool color) {
  Vox<F>::store(geo, i, s, w);
  if (color) {
    uint32_t code = 0;
    if (c3)
      for (int ch = 0; ch < 3; ++ch) code |= (uint32_t)c3[ch] << (8 * ch);
    Vox<F>::store_color(rgb, wc, i, code, cw);
  }
}

template <int F>
void host_load(const void* geo, const uint32_t* rgb, const float* wc, size_t i, float& s,
               float& w, uint32_t& code, float& cw, bool color) {
  Vox<F>::load(geo, i, s, w);
  code = 0;
  cw = 0.f;
  if (color) Vox<F>::load_color(rgb, wc, i, code, cw);
}

dtsdf_status zero_pool(dtsdf_map* m) {
  size_t nv = (size_t)m->p.brick_capacity * kVox;
  DTSDF_HIP(hipMemset(m->geo, 0, nv * geo_bytes(m->fmt)));
  // 0x7f7f7f7f = 3.4e38: a brick without observed voxels bounds nothing
  DTSDF_HIP(hipMemset(m->sub_min, 0x7f, sizeof(float) * 8 * m->p.brick_capacity));
  DTSDF_HIP(hipMemset(m->brick_neg, 0, sizeof(uint64_t) * 16 * m->p.brick_capacity));
  if (m->rgb) DTSDF_HIP(hipMemset(m->rgb, 0, nv * sizeof(uint32_t)));
  if (m->wc) DTSDF_HIP(hipMemset(m->wc, 0, nv * sizeof(float)));
  return DTSDF_OK;
}

}  // namespace

extern "C" {

const char* dtsdf_status_string(dtsdf_status s) {
  switch (s) {
    case DTSDF_OK: return "ok";
    case DTSDF_E_INVAL: return "invalid argument";
    case DTSDF_E_NOMEM: return "out of memory";
    case DTSDF_E_CAPACITY: return "brick pool or hash table full";
    case DTSDF_E_HIP: return "HIP runtime error";
    case DTSDF_E_DEGENERATE: return "degenerate registration problem";
    case DTSDF_E_BUSY: return "busy";
  }
  return "unknown status";
}

dtsdf_status dtsdf_create(const dtsdf_params* p, dtsdf_map** out) {
  if (!p || !out) return DTSDF_E_INVAL;
  *out = nullptr;
  const double kPi = 3.14159265358979323846;
  if (!(p->voxel_size > 0) || !(p->truncation > 0) || !(p->lattice_step > 0)) return DTSDF_E_INVAL;
  if (!(p->theta > 0.25 * kPi + 1e-6) || !(p->theta <= 0.5 * kPi + 1e-6)) return DTSDF_E_INVAL;
  if (!(p->w_max > 0) || p->w_carve < 0 || p->w_min < 0) return DTSDF_E_INVAL;
  if (p->hash_buckets < 2 || (p->hash_buckets & (p->hash_buckets - 1)) != 0) return DTSDF_E_INVAL;
  if (p->brick_capacity == 0 || p->brick_capacity > (1u << 28)) return DTSDF_E_INVAL;
  if (storage_format(*p) < 0) return DTSDF_E_INVAL;
  dtsdf_map* m = new (std::nothrow) dtsdf_map();
  if (!m) return DTSDF_E_NOMEM;
  std::memset(m, 0, sizeof(*m));
  m->p = *p;
  m->fmt = storage_format(*p);
  m->buckets = p->hash_buckets;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return DTSDF_E_HIP;
  }
  size_t nv = (size_t)p->brick_capacity * kVox;
  bool ok = hipMalloc(&m->entries, sizeof(HashEntry) * m->buckets) == hipSuccess &&
            hipMalloc(&m->req, sizeof(uint32_t) * m->buckets) == hipSuccess &&
            hipMalloc(&m->bkey, sizeof(int4) * p->brick_capacity) == hipSuccess &&
            hipMalloc(&m->geo, geo_bytes(m->fmt) * nv) == hipSuccess &&
            hipMalloc(&m->counters, sizeof(int32_t) * 16) == hipSuccess &&
            hipMalloc(&m->vis_list, sizeof(int32_t) * p->brick_capacity) == hipSuccess &&
            hipMalloc(&m->sub_min, sizeof(float) * 8 * p->brick_capacity) == hipSuccess &&
            hipMalloc(&m->slot_min, sizeof(float) * 8 * (size_t)m->buckets) == hipSuccess &&
            hipMalloc(&m->brick_neg, sizeof(uint64_t) * 16 * p->brick_capacity) == hipSuccess &&
            hipMalloc(&m->block_neg, sizeof(uint64_t) * 8 * (size_t)m->buckets) == hipSuccess;
  if (ok && p->with_color) {
    ok = hipMalloc(&m->rgb, sizeof(uint32_t) * nv) == hipSuccess;
    if (ok && m->fmt == 0) ok = hipMalloc(&m->wc, sizeof(float) * nv) == hipSuccess;
  }
  if (!ok) {
    free_map(m);
    return DTSDF_E_NOMEM;
  }
  dtsdf_status st = zero_pool(m);
  if (st == DTSDF_OK && hipMemset(m->req, 0, sizeof(uint32_t) * m->buckets) != hipSuccess)
    st = DTSDF_E_HIP;
  std::vector<HostKey> keys;
  if (st == DTSDF_OK && p->dense) {
    for (int bx = p->dense_lo[0]; bx <= p->dense_hi[0]; ++bx)
      for (int by = p->dense_lo[1]; by <= p->dense_hi[1]; ++by)
        for (int bz = p->dense_lo[2]; bz <= p->dense_hi[2]; ++bz)
          for (int d = 0; d < 6; ++d) keys.push_back(HostKey{bx, by, bz, d});
    if (keys.size() > p->brick_capacity || keys.empty()) st = DTSDF_E_INVAL;
  }
  if (st == DTSDF_OK) st = upload_table(m, keys);
  if (st == DTSDF_OK) st = rebuild_index(m, nullptr);
  if (st == DTSDF_OK && hipDeviceSynchronize() != hipSuccess) st = DTSDF_E_HIP;
  if (st != DTSDF_OK) {
    free_map(m);
    return st;
  }
  *out = m;
  return DTSDF_OK;
}

dtsdf_status dtsdf_destroy(dtsdf_map* m) {
  if (!m) return DTSDF_OK;
  (void)hipDeviceSynchronize();
  free_map(m);
  return DTSDF_OK;
}

dtsdf_status dtsdf_get_info(const dtsdf_map* m, dtsdf_info* out) {
  if (!m || !out) return DTSDF_E_INVAL;
  out->bricks = m->n_bricks - m->n_free;
  out->capacity = m->p.brick_capacity;
  out->blocks = m->n_blocks;
  out->hash_buckets = m->buckets;
  out->dropped = m->dropped;
  size_t nv = (size_t)m->p.brick_capacity * kVox;
  out->device_bytes = (int64_t)(sizeof(HashEntry) * m->buckets + sizeof(uint32_t) * m->buckets +
                                (sizeof(int4) + 8 * sizeof(float) + 16 * sizeof(uint64_t)) *
                                    m->p.brick_capacity +
                                (8 * sizeof(float) + 8 * sizeof(uint64_t)) * m->buckets +
                                geo_bytes(m->fmt) * nv +
                                (m->p.with_color ? (sizeof(uint32_t) + (m->fmt == 0 ? sizeof(float) : 0)) * nv : 0) +
                                (sizeof(GridRec) + 8 * sizeof(uint64_t) + 64) * m->grid_cap +
                                m->mip_cap +
                                (m->free_list ? sizeof(int32_t) * m->p.brick_capacity : 0) +
                                sizeof(int32_t) * m->p.brick_capacity);
  return DTSDF_OK;
}

dtsdf_status dtsdf_export(const dtsdf_map* m, dtsdf_blob* b) {
  if (!m || !b) return DTSDF_E_INVAL;
  if (hipDeviceSynchronize() != hipSuccess) return DTSDF_E_HIP;
  // the pool holds n_bricks slots of which n_free are recycled (direction -1)
  int64_t n = m->n_bricks;
  const int64_t live = m->n_bricks - m->n_free;
  if (!b->keys) {
    b->n_bricks = live;
    return DTSDF_OK;
  }
  if (b->n_bricks < live || !b->sdf || !b->w) return DTSDF_E_INVAL;
  std::vector<int4> bk((size_t)n);
  const size_t gb = geo_bytes(m->fmt);
  std::vector<uint8_t> geo((size_t)n * kVox * gb);
  std::vector<uint32_t> rgb;
  std::vector<float> wc;
  const bool color = m->p.with_color != 0;
  if (n > 0) {
    DTSDF_HIP(hipMemcpy(bk.data(), m->bkey, sizeof(int4) * n, hipMemcpyDeviceToHost));
    DTSDF_HIP(hipMemcpy(geo.data(), m->geo, gb * n * kVox, hipMemcpyDeviceToHost));
    if (color) {
      rgb.resize((size_t)n * kVox);
      DTSDF_HIP(hipMemcpy(rgb.data(), m->rgb, sizeof(uint32_t) * n * kVox, hipMemcpyDeviceToHost));
      if (m->fmt == 0) {
        wc.resize((size_t)n * kVox);
        DTSDF_HIP(hipMemcpy(wc.data(), m->wc, sizeof(float) * n * kVox, hipMemcpyDeviceToHost));
      }
    }
  }
  std::vector<int64_t> order;
  order.reserve((size_t)live);
  for (int64_t i = 0; i < n; ++i)
    if (bk[i].w >= 0) order.push_back(i);
  if ((int64_t)order.size() != live) return DTSDF_E_HIP;
  n = live;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t c) {
    HostKey ka{bk[a].x, bk[a].y, bk[a].z, bk[a].w}, kc{bk[c].x, bk[c].y, bk[c].z, bk[c].w};
    return key_less(ka, kc);
  });
  for (int64_t j = 0; j < n; ++j) {
    int64_t i = order[j];
    b->keys[4 * j + 0] = bk[i].x;
    b->keys[4 * j + 1] = bk[i].y;
    b->keys[4 * j + 2] = bk[i].z;
    b->keys[4 * j + 3] = bk[i].w;
    for (int l = 0; l < kVox; ++l) {
      const size_t src = (size_t)i * kVox + l, dst = (size_t)j * kVox + l;
      float sd, w, cw;
      uint32_t c;
      if (m->fmt == 0)
        host_load<0>(geo.data(), rgb.data(), wc.data(), src, sd, w, c, cw, color);
      else if (m->fmt == 1)
        host_load<1>(geo.data(), rgb.data(), wc.data(), src, sd, w, c, cw, color);
      else
        host_load<2>(geo.data(), rgb.data(), wc.data(), src, sd, w, c, cw, color);
      b->sdf[dst] = sd;
      b->w[dst] = w;
      if (b->rgb)
        for (int ch = 0; ch < 3; ++ch) b->rgb[dst * 3 + ch] = (c >> (8 * ch)) & 0xFF;
      if (b->wc) b->wc[dst] = cw;
    }
  }
  b->n_bricks = n;
  return DTSDF_OK;
}

dtsdf_status dtsdf_import(dtsdf_map* m, const dtsdf_blob* b) {
  if (!m || !b || b->n_bricks < 0 || (b->n_bricks > 0 && (!b->keys || !b->sdf || !b->w)))
    return DTSDF_E_INVAL;
  int64_t n = b->n_bricks;
  if (n > (int64_t)m->p.brick_capacity) return DTSDF_E_CAPACITY;
  if (hipDeviceSynchronize() != hipSuccess) return DTSDF_E_HIP;
  std::vector<HostKey> keys((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    keys[i] = HostKey{b->keys[4 * i], b->keys[4 * i + 1], b->keys[4 * i + 2], b->keys[4 * i + 3]};
    if (m->regular && keys[i].d != 0) return DTSDF_E_INVAL;
  }
  m->mirrored = -1;
  std::vector<int64_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int64_t a, int64_t c) { return key_less(keys[a], keys[c]); });
  std::vector<HostKey> sorted((size_t)n);
  const size_t gb = geo_bytes(m->fmt);
  const bool color = m->p.with_color != 0;
  std::vector<uint8_t> geo((size_t)n * kVox * gb);
  std::vector<uint32_t> rgb(color ? (size_t)n * kVox : 0);
  std::vector<float> wc(color && m->fmt == 0 ? (size_t)n * kVox : 0);
  for (int64_t j = 0; j < n; ++j) {
    int64_t i = order[j];
    sorted[j] = keys[i];
    for (int l = 0; l < kVox; ++l) {
      const size_t src = (size_t)i * kVox + l, dst = (size_t)j * kVox + l;
      const float sd = b->sdf[src], w = b->w[src];
      const uint8_t* c3 = b->rgb ? &b->rgb[src * 3] : nullptr;
      const float cw = b->wc ? b->wc[src] : 0.f;
      if (m->fmt == 0)
        host_store<0>(geo.data(), rgb.data(), wc.data(), dst, sd, w, c3, cw, color);
      else if (m->fmt == 1)
        host_store<1>(geo.data(), rgb.data(), wc.data(), dst, sd, w, c3, cw, color);
      else
        host_store<2>(geo.data(), rgb.data(), wc.data(), dst, sd, w, c3, cw, color);
    }
  }
  dtsdf_status st = zero_pool(m);
  if (st != DTSDF_OK) return st;
  st = upload_table(m, sorted);
  if (st != DTSDF_OK) {
    // leave a consistent empty map behind
    std::vector<HostKey> none;
    upload_table(m, none);
    return st;
  }
  if (n > 0) {
    DTSDF_HIP(hipMemcpy(m->geo, geo.data(), gb * n * kVox, hipMemcpyHostToDevice));
    if (color) {
      DTSDF_HIP(hipMemcpy(m->rgb, rgb.data(), sizeof(uint32_t) * n * kVox, hipMemcpyHostToDevice));
      if (m->fmt == 0)
        DTSDF_HIP(hipMemcpy(m->wc, wc.data(), sizeof(float) * n * kVox, hipMemcpyHostToDevice));
    }
  }
  DTSDF_HIP(hipMemset(m->req, 0, sizeof(uint32_t) * m->buckets));
  st = brick_stats(m, nullptr);
  // the previous contents may have covered blocks the new table does not hold
  if (st == DTSDF_OK) st = rebuild_index_cleared(m, nullptr);
  if (st != DTSDF_OK) return st;
  DTSDF_HIP(hipDeviceSynchronize());
  return DTSDF_OK;
}

}  // extern "C"
