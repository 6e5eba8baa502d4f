// Ray-cast rendering of the Directional TSDF (Sec. 4).
//
// One thread per pixel, 8x8 pixel tiles per wave so that the rays of a wave traverse the same
// bricks.  Per ray:
//   * lattice t_k = t0 + k * step from z_near to z_far (Sec. 4: probing at regular intervals);
//     sample positions are float64 so that the cell a sample falls in is the exact one,
//     interpolation and combination are float32;
//   * a sample whose base voxel lies in a block absent from the hash is undefined in every
//     direction, so the march jumps to the last lattice point before the block exit (exact);
//   * per present direction: trilinear Phi^D, W^D and the analytic gradient of the interpolant
//     over the 8 corners (all corners allocated with W > 0, else the direction is undefined);
//     combination weight w_dir(n^D) max(0, <n^D, -r>) W^D (eq. combine_weight) and the
//     gradient-free fallback W^D max(0, <v^D, -r>) (eq. combine_tsdf_weight);
//   * hit: first k >= 1 with f(t_{k-1}) > 0 >= f(t_k), both defined; the bracket is refined
//     with the Illinois variant of regula falsi (every fourth step a bisection), undefined
//     points counting as free space; outputs are evaluated at the bracket end inside the
//     surface.
#include <cmath>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

struct RenderArgs {
  int W, H;
  double fx, fy, cx, cy;
  double R[9], t[3];
  double z_near, z_far;
  float* depth;
  float* vertex;
  float* normal;
  uint8_t* rgba;
  uint8_t* mask;
  uint8_t* trace_bricks;
  uint8_t* trace_color;
  uint8_t* trace_slots;
};

struct Trace {
  uint8_t* bricks;
  uint8_t* color;
  uint8_t* slots;
};

struct BlockCache {
  int bx, by, bz;
  int slot;
};

__device__ inline int lookup_block(const MapView& m, int bx, int by, int bz, const Trace& tr) {
  if (!key_in_range(bx, by, bz)) return -1;
  const uint64_t key = pack_key(bx, by, bz);
  if (tr.slots) {   // traffic accounting: mark every probed bucket
    uint32_t s = hash_key(key) & m.mask;
    for (uint32_t i = 0; i <= m.mask; ++i) {
      tr.slots[s] = 1;
      uint64_t k = m.entries[s].key;
      if (k == key) return (int)s;
      if (k == kEmptyKey) return -1;
      s = (s + 1) & m.mask;
    }
    return -1;
  }
  return find_slot(m.entries, m.mask, key);
}

struct Eval {
  bool defined;
  bool fallback;
  float f;
  float n[3];       // FULL: sum of omega * (n^D or v^D)
  float rgb[3];     // FULL: combined colour
  bool color_ok;
};

// Evaluates the combined SDF at world point x for unit ray direction r.
// Returns false if the block of the base voxel is absent (the sample is undefined and so
// is every sample in that block); `bc` caches the base block's hash slot.
template <bool FULL>
__device__ bool eval_at(const MapView& m, const double x[3], const float r[3], BlockCache& bc,
                        Eval& e, const Trace& tr) {
  e.defined = false;
  e.fallback = false;
  e.f = 0.f;
  int ix[3], bl[3], lo[3];
  float a[3];
  for (int k = 0; k < 3; ++k) {
    double vx = x[k] * m.inv_voxel;
    double fl = floor(vx);
    ix[k] = (int)fl;
    a[k] = (float)(vx - fl);
    bl[k] = ix[k] >> 3;
    lo[k] = ix[k] & 7;
  }
  if (bl[0] != bc.bx || bl[1] != bc.by || bl[2] != bc.bz) {
    bc.bx = bl[0];
    bc.by = bl[1];
    bc.bz = bl[2];
    bc.slot = lookup_block(m, bl[0], bl[1], bl[2], tr);
  }
  if (bc.slot < 0) return false;
  // hash slots of the blocks the eight corners fall in, indexed by block offset bits
  const int need = (lo[0] == 7 ? 1 : 0) | (lo[1] == 7 ? 2 : 0) | (lo[2] == 7 ? 4 : 0);
  int nb[8];
  nb[0] = bc.slot;
#pragma unroll
  for (int o = 1; o < 8; ++o) {
    nb[o] = -1;
    if ((o & need) == o)
      nb[o] = lookup_block(m, bl[0] + (o & 1), bl[1] + ((o >> 1) & 1), bl[2] + ((o >> 2) & 1), tr);
  }
  int loc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int cx = lo[0] + (c & 1), cy = lo[1] + ((c >> 1) & 1), cz = lo[2] + ((c >> 2) & 1);
    loc[c] = (cx & 7) + 8 * (cy & 7) + 64 * (cz & 7);
  }
  const HashEntry& base = m.entries[bc.slot];
  const float mr[3] = {-r[0], -r[1], -r[2]};
  float phi[6], W[6], om[6], nn[6][3];
  bool def[6], gok[6];
  int brick_of[6][8];
  bool any = false;
  float sum_o = 0.f, sum_op = 0.f;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    def[d] = false;
    gok[d] = false;
    om[d] = 0.f;
    int b0 = base.brick[d];
    if (b0 < 0) continue;
    float sv[8], wv[8];
    bool ok = true;
    for (int c = 0; c < 8 && ok; ++c) {
      int o = c & need;
      int br = b0;
      if (o) {
        int s = nb[o];
        br = s < 0 ? -1 : m.entries[s].brick[d];
      }
      if (br < 0) {
        ok = false;
        break;
      }
      brick_of[d][c] = br;
      if (tr.bricks) tr.bricks[br] = 1;
      float2 v = m.sw[(size_t)br * kVox + loc[c]];
      sv[c] = v.x;
      wv[c] = v.y;
      if (!(v.y > 0.f)) ok = false;
    }
    if (!ok) continue;
    def[d] = true;
    any = true;
    const float ax = a[0], ay = a[1], az = a[2];
    const float bx = 1.f - ax, by = 1.f - ay, bz = 1.f - az;
    // trilinear weights of corners c = (cx, cy, cz)
    const float t0 = bx * by * bz, t1 = ax * by * bz, t2 = bx * ay * bz, t3 = ax * ay * bz;
    const float t4 = bx * by * az, t5 = ax * by * az, t6 = bx * ay * az, t7 = ax * ay * az;
    phi[d] = t0 * sv[0] + t1 * sv[1] + t2 * sv[2] + t3 * sv[3] + t4 * sv[4] + t5 * sv[5] +
             t6 * sv[6] + t7 * sv[7];
    W[d] = t0 * wv[0] + t1 * wv[1] + t2 * wv[2] + t3 * wv[3] + t4 * wv[4] + t5 * wv[5] +
           t6 * wv[6] + t7 * wv[7];
    // analytic gradient of the interpolant (per voxel)
    const float gx = (sv[1] - sv[0]) * by * bz + (sv[3] - sv[2]) * ay * bz +
                     (sv[5] - sv[4]) * by * az + (sv[7] - sv[6]) * ay * az;
    const float gy = (sv[2] - sv[0]) * bx * bz + (sv[3] - sv[1]) * ax * bz +
                     (sv[6] - sv[4]) * bx * az + (sv[7] - sv[5]) * ax * az;
    const float gz = (sv[4] - sv[0]) * bx * by + (sv[5] - sv[1]) * ax * by +
                     (sv[6] - sv[2]) * bx * ay + (sv[7] - sv[3]) * ax * ay;
    const float gl = sqrtf(gx * gx + gy * gy + gz * gz);
    if (gl >= 1e-6f) {
      gok[d] = true;
      const float il = 1.f / gl;
      nn[d][0] = gx * il;
      nn[d][1] = gy * il;
      nn[d][2] = gz * il;
      const float wd = w_dir_cos(axis_dot(nn[d][0], nn[d][1], nn[d][2], d), m.theta);
      const float cs = nn[d][0] * mr[0] + nn[d][1] * mr[1] + nn[d][2] * mr[2];
      om[d] = wd * fmaxf(0.f, cs) * W[d];
    }
    sum_o += om[d];
    sum_op += om[d] * phi[d];
  }
  if (!any) return true;
  if (sum_o > 0.f) {
    e.defined = true;
    e.f = sum_op / sum_o;
  } else {
    // no usable gradient weight in any direction: eq. combine_tsdf_weight
    e.fallback = true;
    sum_o = 0.f;
    sum_op = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      om[d] = 0.f;
      if (!def[d]) continue;
      om[d] = W[d] * fmaxf(0.f, axis_dot(mr[0], mr[1], mr[2], d));
      sum_o += om[d];
      sum_op += om[d] * phi[d];
    }
    if (sum_o > 0.f) {
      e.defined = true;
      e.f = sum_op / sum_o;
    }
  }
  if (FULL) {
    e.n[0] = e.n[1] = e.n[2] = 0.f;
    e.color_ok = false;
    e.rgb[0] = e.rgb[1] = e.rgb[2] = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!def[d] || !(om[d] > 0.f)) continue;
      for (int k = 0; k < 3; ++k) {
        float comp = e.fallback ? ((k == (d >> 1)) ? ((d & 1) ? -1.f : 1.f) : 0.f) : nn[d][k];
        e.n[k] += om[d] * comp;
      }
    }
    if (m.with_color) {
      // colour: per direction trilinear colour over corners with w_c > 0, blended with
      // w_dir(n^D) max(0, <n^D, -r>) W_c^D; if those sum to zero, with the geometric weights
      float cw[6], col[6][3];
      bool cok[6];
      const float ax = a[0], ay = a[1], az = a[2];
      const float bx = 1.f - ax, by = 1.f - ay, bz = 1.f - az;
      const float tw[8] = {bx * by * bz, ax * by * bz, bx * ay * bz, ax * ay * bz,
                           bx * by * az, ax * by * az, bx * ay * az, ax * ay * az};
      for (int d = 0; d < 6; ++d) {
        cok[d] = false;
        if (!def[d]) continue;
        float wsum = 0.f, c3[3] = {0.f, 0.f, 0.f};
        bool ok = true;
        for (int c = 0; c < 8; ++c) {
          size_t vi = (size_t)brick_of[d][c] * kVox + loc[c];
          if (tr.color) tr.color[brick_of[d][c]] = 1;
          float w = m.wc[vi];
          if (!(w > 0.f)) {
            ok = false;
            break;
          }
          uint32_t code = m.rgb[vi];
          wsum += tw[c] * w;
          for (int ch = 0; ch < 3; ++ch) c3[ch] += tw[c] * (float)((code >> (8 * ch)) & 0xFFu);
        }
        if (!ok) continue;
        cok[d] = true;
        cw[d] = wsum;
        for (int ch = 0; ch < 3; ++ch) col[d][ch] = c3[ch];
      }
      float so = 0.f, sc[3] = {0.f, 0.f, 0.f};
      if (!e.fallback)
        for (int d = 0; d < 6; ++d) {
          if (!cok[d] || !gok[d]) continue;
          float oc = w_dir_cos(axis_dot(nn[d][0], nn[d][1], nn[d][2], d), m.theta) *
                     fmaxf(0.f, nn[d][0] * mr[0] + nn[d][1] * mr[1] + nn[d][2] * mr[2]) * cw[d];
          so += oc;
          for (int ch = 0; ch < 3; ++ch) sc[ch] += oc * col[d][ch];
        }
      if (!(so > 0.f)) {
        so = 0.f;
        sc[0] = sc[1] = sc[2] = 0.f;
        for (int d = 0; d < 6; ++d) {
          if (!cok[d]) continue;
          so += om[d];
          for (int ch = 0; ch < 3; ++ch) sc[ch] += om[d] * col[d][ch];
        }
      }
      if (so > 0.f) {
        e.color_ok = true;
        for (int ch = 0; ch < 3; ++ch) e.rgb[ch] = sc[ch] / so;
      }
    }
  }
  return true;
}

__global__ __launch_bounds__(64) void render_k(MapView m, RenderArgs a) {
  const int u = blockIdx.x * 8 + (threadIdx.x & 7);
  const int v = blockIdx.y * 8 + (threadIdx.x >> 3);
  if (u >= a.W || v >= a.H) return;
  const size_t i = (size_t)v * a.W + u;
  const size_t HW = (size_t)a.W * a.H;
  double dc[3] = {((double)u - a.cx) / a.fx, ((double)v - a.cy) / a.fy, 1.0};
  const double len = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
  const double rc[3] = {dc[0] / len, dc[1] / len, dc[2] / len};
  double r[3];
  for (int k = 0; k < 3; ++k) r[k] = a.R[3 * k] * rc[0] + a.R[3 * k + 1] * rc[1] + a.R[3 * k + 2] * rc[2];
  const float rf[3] = {(float)r[0], (float)r[1], (float)r[2]};
  const double* o = a.t;
  const double t0 = a.z_near / rc[2], tmax = a.z_far / rc[2];
  const double step = m.step;
  BlockCache bc{0x7fffffff, 0, 0, -1};
  const Trace tr{a.trace_bricks, a.trace_color, a.trace_slots};
  bool prev_def = false, hit = false;
  float prev_f = 0.f, fa = 0.f, fb = 0.f;
  double ta = 0.0, tb = 0.0;
  for (long long k = 0;;) {
    const double tk = t0 + (double)k * step;
    if (tk > tmax) break;
    const double x[3] = {o[0] + tk * r[0], o[1] + tk * r[1], o[2] + tk * r[2]};
    Eval e;
    if (!eval_at<false>(m, x, rf, bc, e, tr)) {
      // every lattice point before the exit of this absent block is undefined
      double texit = 1e300;
      for (int ax = 0; ax < 3; ++ax) {
        int b = ax == 0 ? bc.bx : (ax == 1 ? bc.by : bc.bz);
        if (r[ax] > 0.0) texit = fmin(texit, ((double)(b + 1) * kB * m.voxel - o[ax]) / r[ax]);
        else if (r[ax] < 0.0) texit = fmin(texit, ((double)b * kB * m.voxel - o[ax]) / r[ax]);
      }
      const double jn = ceil((texit - 1e-6 - t0) / step);
      long long j0 = jn > 9e15 ? (long long)9e15 : (long long)jn;
      k = j0 > k + 1 ? j0 : k + 1;
      prev_def = false;
      continue;
    }
    if (k >= 1 && e.defined && prev_def && prev_f > 0.f && e.f <= 0.f) {
      hit = true;
      ta = t0 + (double)(k - 1) * step;
      tb = tk;
      fa = prev_f;
      fb = e.f;
      break;
    }
    prev_def = e.defined;
    prev_f = e.f;
    ++k;
  }
  float out_depth = 0.f, out_v[3] = {0.f, 0.f, 0.f}, out_n[3] = {0.f, 0.f, 0.f};
  uint32_t out_c = 0;
  if (hit) {
    int side = 0;
    for (int it = 0; it < 40 && (tb - ta) > 1e-7; ++it) {
      double c = (it & 3) == 3 ? 0.5 * (ta + tb)
                               : ta + (tb - ta) * ((double)fa / ((double)fa - (double)fb));
      if (!(c > ta && c < tb)) c = 0.5 * (ta + tb);
      const double x[3] = {o[0] + c * r[0], o[1] + c * r[1], o[2] + c * r[2]};
      Eval e;
      bool present = eval_at<false>(m, x, rf, bc, e, tr);
      if (!present || !e.defined || e.f > 0.f) {
        ta = c;
        if (present && e.defined) fa = e.f;
        if (side == 1) fb *= 0.5f;
        side = 1;
      } else {
        tb = c;
        fb = e.f;
        if (side == -1) fa *= 0.5f;
        side = -1;
      }
    }
    const double ts = 0.5 * (ta + tb);
    const double x[3] = {o[0] + tb * r[0], o[1] + tb * r[1], o[2] + tb * r[2]};
    Eval e;
    eval_at<true>(m, x, rf, bc, e, tr);
    out_depth = (float)(ts * rc[2]);
    for (int k = 0; k < 3; ++k) out_v[k] = (float)(ts * rc[k]);
    const float nl = sqrtf(e.n[0] * e.n[0] + e.n[1] * e.n[1] + e.n[2] * e.n[2]);
    if (nl > 0.f) {
      for (int k = 0; k < 3; ++k)   // world -> camera: R^T n
        out_n[k] = (float)((a.R[k] * e.n[0] + a.R[3 + k] * e.n[1] + a.R[6 + k] * e.n[2]) / nl);
    }
    if (m.with_color && e.color_ok) {
      out_c = 0xFF000000u;
      for (int ch = 0; ch < 3; ++ch) {
        float q = fminf(255.f, fmaxf(0.f, rintf(e.rgb[ch])));
        out_c |= (uint32_t)q << (8 * ch);
      }
    }
  }
  if (a.depth) a.depth[i] = out_depth;
  if (a.vertex) {
    a.vertex[i] = out_v[0];
    a.vertex[HW + i] = out_v[1];
    a.vertex[2 * HW + i] = out_v[2];
  }
  if (a.normal) {
    a.normal[i] = out_n[0];
    a.normal[HW + i] = out_n[1];
    a.normal[2 * HW + i] = out_n[2];
  }
  if (a.rgba) reinterpret_cast<uint32_t*>(a.rgba)[i] = out_c;
  if (a.mask) a.mask[i] = hit ? 1 : 0;
}

}  // namespace

extern "C" dtsdf_status dtsdf_render(const dtsdf_map* m, const dtsdf_intrinsics* intr,
                                     const double T[16], float z_near, float z_far,
                                     const dtsdf_render_out* out, void* stream) {
  if (!m || !intr || !T || !out || intr->width <= 0 || intr->height <= 0 || intr->width > 16384 ||
      intr->height > 16384 || !(intr->fx > 0) || !(intr->fy > 0) || !(z_near > 0) ||
      !(z_far > z_near))
    return DTSDF_E_INVAL;
  if (out->rgba && ((uintptr_t)out->rgba & 3u)) return DTSDF_E_INVAL;
  RenderArgs a;
  a.W = intr->width;
  a.H = intr->height;
  a.fx = intr->fx;
  a.fy = intr->fy;
  a.cx = intr->cx;
  a.cy = intr->cy;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) a.R[3 * r + c] = T[4 * r + c];
    a.t[r] = T[4 * r + 3];
  }
  a.z_near = (double)z_near;
  a.z_far = (double)z_far;
  a.depth = out->depth;
  a.vertex = out->vertex;
  a.normal = out->normal;
  a.rgba = out->rgba;
  a.mask = out->mask;
  a.trace_bricks = out->trace_bricks;
  a.trace_color = out->trace_color;
  a.trace_slots = out->trace_slots;
  dim3 grd((a.W + 7) / 8, (a.H + 7) / 8);
  hipLaunchKernelGGL(render_k, grd, dim3(64), 0, (hipStream_t)stream, make_view(m), a);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}
