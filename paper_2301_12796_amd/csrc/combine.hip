// View-dependent combined ("rendering") TSDF and conditional recombination (Sec. 4: Lemma
// positional_unambiguity, the precomputed combined TSDF, eq. condition_1 .. condition_4;
// Sec. 7: evaluation at integer voxel positions with six-neighbour gradients, the source
// block and its face neighbours staged in on-chip memory).
//
// The combined TSDF is a regular map (`regular` set) whose direction slot 0 holds, per voxel,
// the combined SDF of the six directions for one camera centre, weight 1 where it is defined
// and 0 where it holds no value, and the combined colour.  It is rendered by the ordinary
// ray march without direction weighting, so one lattice sample reads 8 voxels of one volume
// instead of 8 per allocated direction.
//
// Per call:
//   1. mirror_k   (only when the source gained blocks) every source block gets its brick in
//                 the volume: keys inserted by CAS, pool indices handed out by the allocator
//   2. combine_k  one workgroup per volume brick, 256 threads x 2 voxels: a conservative
//                 box-frustum test per block, then per allocated source direction the brick
//                 plus its six 8x8 face slices staged in LDS, central differences, weights of
//                 eq. combine_weight (fallback eq. combine_tsdf_weight), the colour blend, and
//                 the brick's summaries for the render index
//   3. index update of the volume (occupancy grid, positive cells, direction groups)
#include <cmath>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

struct Frus {
  double R[9], t[3];                 // camera -> world of the frustum's pose
  double fx, fy, cx, cy;
  double umin, umax, vmin, vmax;     // accepted projections [umin, umax) x [vmin, vmax)
  double L[5][3];                    // world gradients of the five half-space forms
};

struct CombArgs {
  Frus F;
  double c[3];                       // camera centre of the combination
  int only_missing;
};

// Whether world point x lies in front of the camera and projects into the widened image.
__device__ inline bool frus_inside(const Frus& F, double x0, double x1, double x2) {
  const double d0 = x0 - F.t[0], d1 = x1 - F.t[1], d2 = x2 - F.t[2];
  const double y0 = F.R[0] * d0 + F.R[3] * d1 + F.R[6] * d2;
  const double y1 = F.R[1] * d0 + F.R[4] * d1 + F.R[7] * d2;
  const double y2 = F.R[2] * d0 + F.R[5] * d1 + F.R[8] * d2;
  if (!(y2 > 0.0)) return false;
  const double u = F.fx * y0 / y2 + F.cx, v = F.fy * y1 / y2 + F.cy;
  return u >= F.umin && u < F.umax && v >= F.vmin && v < F.vmax;
}

// True if no point of the box [lo, hi] can pass frus_inside: some half-space form
// (z > 0, u >= umin, u < umax, v >= vmin, v < vmax, each linear in x) stays below -1e-6 over
// the whole box.  Exact up to that margin, far above the rounding of either evaluation.
__device__ inline bool box_outside(const Frus& F, const double lo[3], const double hi[3]) {
  double c[3], h[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.5 * (lo[k] + hi[k]) - F.t[k];
    h[k] = 0.5 * (hi[k] - lo[k]);
  }
  for (int f = 0; f < 5; ++f) {
    const double* g = F.L[f];
    const double mx = g[0] * c[0] + g[1] * c[1] + g[2] * c[2] + fabs(g[0]) * h[0] +
                      fabs(g[1]) * h[1] + fabs(g[2]) * h[2];
    if (mx < -1e-6) return true;
  }
  return false;
}

__global__ __launch_bounds__(256) void mirror_k(const HashEntry* __restrict__ src, uint32_t n,
                                                HashEntry* dst, uint32_t* req, uint32_t mask,
                                                int32_t* counters, int32_t max_entries) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint64_t k = src[s].key;
  if (k == kEmptyKey) return;
  insert_request(dst, req, mask, k, 0, counters, max_entries);
}

// LDS index of voxel (x, y, z), each in [-1, 8], of a brick padded by one voxel per side.
__device__ inline int pad(int x, int y, int z) { return (x + 1) + 10 * (y + 1) + 100 * (z + 1); }

template <int FS>
__global__ __launch_bounds__(256) void combine_k(MapView src, MapView vol, CombArgs a,
                                                 float* __restrict__ sub_min,
                                                 uint64_t* __restrict__ brick_neg) {
  __shared__ float2 sh[1000];
  __shared__ int s_slot[7];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int4 key = vol.bkey[b];
  uint64_t* bn = brick_neg + (size_t)b * 16;
  // observed (valued) voxel words of the volume brick, word z, bit x + 8 y
  bool has = false;
#pragma unroll
  for (int z = 0; z < 8; ++z) has = has || bn[8 + z] != 0;
  const double s = vol.voxel;
  const double lo[3] = {(double)(key.x * kB) * s, (double)(key.y * kB) * s, (double)(key.z * kB) * s};
  const double hi[3] = {lo[0] + 7.0 * s, lo[1] + 7.0 * s, lo[2] + 7.0 * s};
  if (box_outside(a.F, lo, hi)) {
    if (a.only_missing || !has) return;
    for (int l = tid; l < kVox; l += 256) {
      const size_t vi = (size_t)b * kVox + l;
      Vox<0>::store(vol.geo, vi, 0.f, 0.f);
      if (vol.with_color) Vox<0>::store_color(vol.rgb, vol.wc, vi, 0u, 0.f);
    }
    __syncthreads();
    brick_sub_min<0>(vol.geo, b, sub_min + (size_t)b * 8, bn);
    return;
  }
  if (tid < 7) {
    // centre, -x, +x, -y, +y, -z, +z
    const int ax = tid == 0 ? -1 : (tid - 1) >> 1;
    const int sg = ((tid - 1) & 1) ? 1 : -1;
    const int bx = key.x + (ax == 0 ? sg : 0), by = key.y + (ax == 1 ? sg : 0),
              bz = key.z + (ax == 2 ? sg : 0);
    s_slot[tid] = key_in_range(bx, by, bz) ? find_slot(src.entries, src.mask, pack_key(bx, by, bz)) : -1;
  }
  // per-voxel state, voxel l = tid + 256 j
  bool todo[2], clear[2];
  float rx[2], ry[2], rz[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int l = tid + 256 * j;
    const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
    const double x0 = (double)(key.x * kB + lx) * s, x1 = (double)(key.y * kB + ly) * s,
                 x2 = (double)(key.z * kB + lz) * s;
    const bool inside = frus_inside(a.F, x0, x1, x2);
    const bool valued = (bn[8 + lz] >> (lx + 8 * ly)) & 1ull;
    todo[j] = inside && !(a.only_missing && valued);
    clear[j] = !inside && !a.only_missing && valued;
    const double d0 = x0 - a.c[0], d1 = x1 - a.c[1], d2 = x2 - a.c[2];
    const double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double il = len > 0.0 ? 1.0 / len : 0.0;
    rx[j] = (float)(d0 * il);
    ry[j] = (float)(d1 * il);
    rz[j] = (float)(d2 * il);
    todo[j] = todo[j] && len > 0.0;
  }
  __syncthreads();
  const int cs = s_slot[0];
  float sw[2] = {0.f, 0.f};                       // sum of W over observed directions
  float so[2] = {0.f, 0.f}, sop[2] = {0.f, 0.f};  // gradient weights
  float fo[2] = {0.f, 0.f}, fop[2] = {0.f, 0.f};  // fallback weights
  float cgo[2] = {0.f, 0.f}, cggo[2] = {0.f, 0.f}, cgfo[2] = {0.f, 0.f};
  float cg[2][3] = {}, cgg[2][3] = {}, cgf[2][3] = {};
  const bool any_todo = __syncthreads_or(todo[0] || todo[1]);
  if (any_todo && cs >= 0) {
    for (int d = 0; d < 6; ++d) {
      const int cb = src.entries[cs].brick[d];
      if (cb < 0) continue;
      __syncthreads();   // the previous direction's readers are done with sh
      for (int l = tid; l < kVox; l += 256) {
        float sd, w;
        Vox<FS>::load(src.geo, (size_t)cb * kVox + l, sd, w);
        sh[pad(l & 7, (l >> 3) & 7, l >> 6)] = make_float2(sd, w);
      }
      for (int h = tid; h < 384; h += 256) {
        const int f = h >> 6, q = h & 63, p0 = q & 7, p1 = q >> 3;
        // face f: the neighbour's voxel next to the brick and its LDS position
        int sx, sy, sz, dx, dy, dz;
        switch (f) {
          case 0: sx = 7; sy = p0; sz = p1; dx = -1; dy = p0; dz = p1; break;
          case 1: sx = 0; sy = p0; sz = p1; dx = 8; dy = p0; dz = p1; break;
          case 2: sx = p0; sy = 7; sz = p1; dx = p0; dy = -1; dz = p1; break;
          case 3: sx = p0; sy = 0; sz = p1; dx = p0; dy = 8; dz = p1; break;
          case 4: sx = p0; sy = p1; sz = 7; dx = p0; dy = p1; dz = -1; break;
          default: sx = p0; sy = p1; sz = 0; dx = p0; dy = p1; dz = 8; break;
        }
        const int sl = s_slot[1 + f];
        const int nbf = sl >= 0 ? src.entries[sl].brick[d] : -1;
        float sd = 0.f, w = 0.f;
        if (nbf >= 0) Vox<FS>::load(src.geo, (size_t)nbf * kVox + sx + 8 * sy + 64 * sz, sd, w);
        sh[pad(dx, dy, dz)] = make_float2(sd, w);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!todo[j]) continue;
        const int l = tid + 256 * j;
        const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
        const float2 cv = sh[pad(lx, ly, lz)];
        if (!(cv.y > 0.f)) continue;
        const float W = cv.y, phi = cv.x;
        const float2 xm = sh[pad(lx - 1, ly, lz)], xp = sh[pad(lx + 1, ly, lz)];
        const float2 ym = sh[pad(lx, ly - 1, lz)], yp = sh[pad(lx, ly + 1, lz)];
        const float2 zm = sh[pad(lx, ly, lz - 1)], zp = sh[pad(lx, ly, lz + 1)];
        const bool all = xm.y > 0.f && xp.y > 0.f && ym.y > 0.f && yp.y > 0.f && zm.y > 0.f &&
                         zp.y > 0.f;
        // central differences (times 2 s); the gradient is usable if |grad| s >= 1e-6
        const float gx = xp.x - xm.x, gy = yp.x - ym.x, gz = zp.x - zm.x;
        const float gl2 = sqrtf(gx * gx + gy * gy + gz * gz);
        const bool gok = all && 0.5f * gl2 >= 1e-6f;
        const float mr0 = -rx[j], mr1 = -ry[j], mr2 = -rz[j];
        float om = 0.f, wdc = 0.f;
        if (gok) {
          const float il = 1.f / gl2;
          const float n0 = gx * il, n1 = gy * il, n2 = gz * il;
          wdc = w_dir_cos(axis_dot(n0, n1, n2, d), vol.theta) *
                fmaxf(0.f, n0 * mr0 + n1 * mr1 + n2 * mr2);
          om = wdc * W;
        }
        const float fb = W * fmaxf(0.f, axis_dot(mr0, mr1, mr2, d));
        sw[j] += W;
        so[j] += om;
        sop[j] += om * phi;
        fo[j] += fb;
        fop[j] += fb * phi;
        if (vol.with_color && src.with_color) {
          float Wc;
          uint32_t code;
          Vox<FS>::load_color(src.rgb, src.wc, (size_t)cb * kVox + l, code, Wc);
          if (Wc > 0.f) {
            const float c3[3] = {(float)(code & 0xFFu), (float)((code >> 8) & 0xFFu),
                                 (float)((code >> 16) & 0xFFu)};
            const float oc = wdc * Wc;   // w_dir(n^D) max(0, <n^D, -r>) W_c^D
            cgo[j] += oc;
            cggo[j] += om;
            cgfo[j] += fb;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
              cg[j][ch] += oc * c3[ch];
              cgg[j][ch] += om * c3[ch];
              cgf[j][ch] += fb * c3[ch];
            }
          }
        }
      }
    }
  }
  bool wrote = false;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const size_t vi = (size_t)b * kVox + tid + 256 * j;
    if (todo[j]) {
      bool def = false, fall = false;
      float f = 0.f;
      if (sw[j] > 0.f) {
        if (so[j] > 0.f) {
          def = true;
          f = sop[j] / so[j];
        } else {
          // no usable gradient weight in any direction: eq. combine_tsdf_weight
          fall = true;
          if (fo[j] > 0.f) {
            def = true;
            f = fop[j] / fo[j];
          }
        }
      }
      Vox<0>::store(vol.geo, vi, def ? f : 0.f, def ? 1.f : 0.f);
      if (vol.with_color) {
        float c[3] = {cg[j][0], cg[j][1], cg[j][2]};
        float w = cgo[j];
        if (fall) {
          c[0] = cgf[j][0];
          c[1] = cgf[j][1];
          c[2] = cgf[j][2];
          w = cgfo[j];
        } else if (!(w > 0.f)) {
          c[0] = cgg[j][0];
          c[1] = cgg[j][1];
          c[2] = cgg[j][2];
          w = cggo[j];
        }
        uint32_t code = 0;
        const bool cok = def && w > 0.f;
        if (cok) {
          const float iw = 1.f / w;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const float q = fminf(255.f, fmaxf(0.f, rintf(c[ch] * iw)));
            code |= (uint32_t)q << (8 * ch);
          }
        }
        Vox<0>::store_color(vol.rgb, vol.wc, vi, code, cok ? 1.f : 0.f);
      }
      wrote = true;
    } else if (clear[j]) {
      Vox<0>::store(vol.geo, vi, 0.f, 0.f);
      if (vol.with_color) Vox<0>::store_color(vol.rgb, vol.wc, vi, 0u, 0.f);
      wrote = true;
    }
  }
  if (__syncthreads_or(wrote)) brick_sub_min<0>(vol.geo, b, sub_min + (size_t)b * 8, bn);
}

bool valid_intr(const dtsdf_intrinsics* i) {
  return i && i->width > 0 && i->height > 0 && i->width <= 16384 && i->height <= 16384 &&
         i->fx > 0 && i->fy > 0;
}

Frus make_frus(const double T[16], const dtsdf_intrinsics* in, double margin) {
  Frus F;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) F.R[3 * r + c] = T[4 * r + c];
    F.t[r] = T[4 * r + 3];
  }
  F.fx = in->fx;
  F.fy = in->fy;
  F.cx = in->cx;
  F.cy = in->cy;
  // pixel centres at integer coordinates: the image covers [-1/2, W - 1/2), widened by
  // `margin` times its size per side
  F.umin = -0.5 - margin * in->width;
  F.umax = in->width - 0.5 + margin * in->width;
  F.vmin = -0.5 - margin * in->height;
  F.vmax = in->height - 0.5 + margin * in->height;
  // camera-frame forms y2, fx y0 + (cx - umin) y2, (umax - cx) y2 - fx y0, and the same in v;
  // y_j = sum_i R[3 i + j] (x_i - t_i), so each form's world gradient combines columns of R
  const double a[5][3] = {{0.0, 0.0, 1.0},
                          {F.fx, 0.0, F.cx - F.umin},
                          {-F.fx, 0.0, F.umax - F.cx},
                          {0.0, F.fy, F.cy - F.vmin},
                          {0.0, -F.fy, F.vmax - F.cy}};
  for (int f = 0; f < 5; ++f)
    for (int i = 0; i < 3; ++i)
      F.L[f][i] = a[f][0] * F.R[3 * i] + a[f][1] * F.R[3 * i + 1] + a[f][2] * F.R[3 * i + 2];
  return F;
}

// Gives every block of `src` its brick in `vol` (direction slot 0).
dtsdf_status mirror_blocks(const dtsdf_map* src, dtsdf_map* vol, hipStream_t st) {
  const int32_t max_entries = (int32_t)((uint64_t)vol->buckets * 3 / 4);
  hipLaunchKernelGGL(mirror_k, dim3((src->buckets + 255) / 256), dim3(256), 0, st, src->entries,
                     src->buckets, vol->entries, vol->req, vol->buckets - 1, vol->counters,
                     max_entries);
  const dtsdf_status as = launch_assign(vol, st);
  if (as != DTSDF_OK) return as;
  launch_bbox(vol, st);
  int32_t c[10];
  DTSDF_HIP(hipMemcpyAsync(c, vol->counters, sizeof(c), hipMemcpyDeviceToHost, st));
  DTSDF_HIP(hipStreamSynchronize(st));
  dtsdf_status gs = ensure_grid(vol, c + 4, st);
  if (gs != DTSDF_OK) return gs;
  int64_t handed = c[0];
  if (handed > (int64_t)vol->p.brick_capacity) {
    launch_clamp_handed(vol, st);
    handed = vol->p.brick_capacity;
  }
  const bool dropped = c[1] > vol->dropped;
  vol->dropped = c[1];
  vol->n_bricks = handed;
  vol->n_blocks = c[3];
  if (dropped) return DTSDF_E_CAPACITY;
  vol->mirrored = src->n_blocks;
  return DTSDF_OK;
}

}  // namespace

extern "C" {

dtsdf_status dtsdf_volume_create(const dtsdf_map* src, uint32_t brick_capacity,
                                 uint32_t hash_buckets, dtsdf_map** out) {
  if (!src || !out || src->regular) return DTSDF_E_INVAL;
  dtsdf_params p = src->p;
  p.sdf_fmt = DTSDF_SDF_F32;
  p.w_fmt = DTSDF_W_F32;
  p.brick_capacity = brick_capacity;
  p.hash_buckets = hash_buckets;
  p.dense = 0;
  dtsdf_status st = dtsdf_create(&p, out);
  if (st != DTSDF_OK) return st;
  (*out)->regular = 1;
  (*out)->mirrored = -1;
  return DTSDF_OK;
}

dtsdf_status dtsdf_combine(const dtsdf_map* src, dtsdf_map* vol, const double T_center[16],
                           const double T_frustum[16], const dtsdf_intrinsics* intr,
                           float margin, int32_t only_missing, void* stream) {
  if (!src || !vol || src->regular || !vol->regular || !T_center || !T_frustum ||
      !valid_intr(intr) || !(margin >= 0.f) || !(margin <= 4.f))
    return DTSDF_E_INVAL;
  if (src->p.voxel_size != vol->p.voxel_size || src->p.theta != vol->p.theta)
    return DTSDF_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  if (vol->mirrored != src->n_blocks) {
    dtsdf_status ms = mirror_blocks(src, vol, st);
    if (ms != DTSDF_OK) return ms;
  }
  CombArgs a;
  a.F = make_frus(T_frustum, intr, (double)margin);
  for (int k = 0; k < 3; ++k) a.c[k] = T_center[4 * k + 3];
  a.only_missing = only_missing ? 1 : 0;
  if (vol->n_bricks > 0) {
    const dim3 grd((uint32_t)vol->n_bricks);
    const MapView sv = make_view(src), vv = make_view(vol);
    if (src->fmt == 0)
      hipLaunchKernelGGL(combine_k<0>, grd, dim3(256), 0, st, sv, vv, a, vol->sub_min, vol->brick_neg);
    else if (src->fmt == 1)
      hipLaunchKernelGGL(combine_k<1>, grd, dim3(256), 0, st, sv, vv, a, vol->sub_min, vol->brick_neg);
    else
      hipLaunchKernelGGL(combine_k<2>, grd, dim3(256), 0, st, sv, vv, a, vol->sub_min, vol->brick_neg);
    DTSDF_HIP(hipGetLastError());
  }
  return launch_index_update(vol, st);
}

dtsdf_status dtsdf_recombine_decide(dtsdf_recombine_state* s, const double T[16],
                                    int32_t* recombine) {
  if (!s || !T || !recombine) return DTSDF_E_INVAL;
  bool need = !s->has_pose || s->frames < s->boot_frames || s->since > s->stale_frames;
  if (!need) {
    double dt2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double d = T[4 * k + 3] - s->last_pose[4 * k + 3];
      dt2 += d * d;
    }
    // relative rotation R_last^T R: its angle from the trace and the skew part
    double Q[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += s->last_pose[4 * k + i] * T[4 * k + j];
        Q[3 * i + j] = acc;
      }
    const double sx = Q[7] - Q[5], sy = Q[2] - Q[6], sz = Q[3] - Q[1];
    const double angle = atan2(0.5 * sqrt(sx * sx + sy * sy + sz * sz),
                               0.5 * (Q[0] + Q[4] + Q[8] - 1.0));
    need = sqrt(dt2) > s->max_translation || angle > s->max_angle;
  }
  s->frames += 1;
  if (need) {
    s->since = 1;
    for (int k = 0; k < 16; ++k) s->last_pose[k] = T[k];
    s->has_pose = 1;
  } else {
    s->since += 1;
  }
  *recombine = need ? 1 : 0;
  return DTSDF_OK;
}

}  // extern "C"
