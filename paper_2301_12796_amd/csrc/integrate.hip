// Integration of depth (+colour) frames into the Directional TSDF (Sec. 3 and Sec. 7).
//
// Per frame:
//   1. vertex_normal_k   back-projection (eq. reprojection) and cross-product normals of the
//                        depth image, one thread per pixel, float64 arithmetic
//   2. request_k         (sparse maps) block requests along p +/- tau r for every direction
//                        with w_dir > 0, inserted into the spatial hash by CAS
//   3. collect_k,        pool indices for newly requested (block, D) bricks, handed out in
//      assign_sorted_k   sorted (block key, D) order (a radix sort between the two)
//   4. carve_guard_k     the carving guard of every pixel (depth jumps within two pixels)
//   5. cull_k            conservative frustum test per brick: the list of bricks to visit
//   6. fuse_k            voxel-projection fusion of every listed brick, one workgroup per
//                        brick, 256 threads x 2 voxels: HBM streaming of (sdf, w) (+ colour)
// Geometry (projection, point-to-plane distance) is evaluated in float64 so that the
// discrete decisions (pixel association, band tests) match an exact evaluation except on
// measure-zero ties; the running averages are float32, as stored.
#include <algorithm>
#include <cmath>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

struct Intr {
  int W, H;
  double fx, fy, cx, cy;
};

__global__ __launch_bounds__(256) void vertex_normal_k(const float* __restrict__ depth, Intr in,
                                                       double scale, float* __restrict__ vmap,
                                                       float* __restrict__ nmap) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y * blockDim.y + threadIdx.y;
  if (u >= in.W || v >= in.H) return;
  const size_t HW = (size_t)in.W * in.H;
  const size_t i = (size_t)v * in.W + u;
  auto point = [&](int uu, int vv, double* P) -> bool {
    double z = (double)depth[(size_t)vv * in.W + uu] * scale;
    if (!(z > 0.0) || !isfinite(z)) return false;
    P[0] = z * ((double)uu - in.cx) / in.fx;
    P[1] = z * ((double)vv - in.cy) / in.fy;
    P[2] = z;
    return true;
  };
  double P[3] = {0, 0, 0};
  bool pv = point(u, v, P);
  vmap[i] = pv ? (float)P[0] : 0.f;
  vmap[HW + i] = pv ? (float)P[1] : 0.f;
  vmap[2 * HW + i] = pv ? (float)P[2] : 0.f;
  float n_out[3] = {0.f, 0.f, 0.f};
  if (pv && u > 0 && v > 0 && u + 1 < in.W && v + 1 < in.H) {
    double L[3], Rr[3], T[3], B[3];
    if (point(u - 1, v, L) && point(u + 1, v, Rr) && point(u, v - 1, T) && point(u, v + 1, B)) {
      double dx[3] = {Rr[0] - L[0], Rr[1] - L[1], Rr[2] - L[2]};
      double dy[3] = {B[0] - T[0], B[1] - T[1], B[2] - T[2]};
      double n[3] = {dx[1] * dy[2] - dx[2] * dy[1], dx[2] * dy[0] - dx[0] * dy[2],
                     dx[0] * dy[1] - dx[1] * dy[0]};
      double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      if (len > 0.0) {
        double s = (n[0] * P[0] + n[1] * P[1] + n[2] * P[2] > 0.0) ? -1.0 / len : 1.0 / len;
        for (int k = 0; k < 3; ++k) n_out[k] = (float)(n[k] * s);
      }
    }
  }
  nmap[i] = n_out[0];
  nmap[HW + i] = n_out[1];
  nmap[2 * HW + i] = n_out[2];
}

__global__ __launch_bounds__(256) void downsample_k(const float* __restrict__ in, int W, int H,
                                                    float* __restrict__ out) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y * blockDim.y + threadIdx.y;
  int Wo = W / 2, Ho = H / 2;
  if (u >= Wo || v >= Ho) return;
  const float* r0 = in + (size_t)(2 * v) * W + 2 * u;
  const float* r1 = r0 + W;
  float a = r0[0], b = r0[1], c = r1[0], d = r1[1];
  out[(size_t)v * Wo + u] = (a > 0.f && b > 0.f && c > 0.f && d > 0.f) ? (a + b + c + d) * 0.25f : 0.f;
}

struct Pose {
  double R[9];
  double t[3];
};

// Allocation requests (Sec. 7: blocks are allocated for every point with a valid normal):
// for each direction D with w_dir(n) > 0, the blocks containing the J + 1 evenly spaced
// points p + s r, s in [-tau, tau] (r: unit ray through the pixel).
__global__ __launch_bounds__(256) void request_k(const float* __restrict__ depth,
                                                 const float* __restrict__ nmap, Intr in,
                                                 double scale, Pose T, double voxel, double tau,
                                                 int J, float theta, HashEntry* entries,
                                                 uint32_t* req, uint32_t mask,
                                                 int32_t* counters, int32_t max_entries) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y * blockDim.y + threadIdx.y;
  if (u >= in.W || v >= in.H) return;
  const size_t HW = (size_t)in.W * in.H;
  const size_t i = (size_t)v * in.W + u;
  float nx = nmap[i], ny = nmap[HW + i], nz = nmap[2 * HW + i];
  if (nx == 0.f && ny == 0.f && nz == 0.f) return;
  double z = (double)depth[i] * scale;
  if (!(z > 0.0) || !isfinite(z)) return;     // a caller normal on a pixel without depth
  double pc[3] = {z * ((double)u - in.cx) / in.fx, z * ((double)v - in.cy) / in.fy, z};
  double len = sqrt(pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
  double pw[3], rw[3];
  float nw[3];
  for (int k = 0; k < 3; ++k) {
    double rp = T.R[3 * k] * pc[0] + T.R[3 * k + 1] * pc[1] + T.R[3 * k + 2] * pc[2];
    pw[k] = rp + T.t[k];
    rw[k] = rp / len;
    nw[k] = (float)(T.R[3 * k] * nx + T.R[3 * k + 1] * ny + T.R[3 * k + 2] * nz);
  }
  for (int d = 0; d < 6; ++d) {
    if (!(w_dir_cos(axis_dot(nw[0], nw[1], nw[2], d), theta) > 0.f)) continue;
    uint64_t prev = kEmptyKey;
    for (int j = 0; j <= J; ++j) {
      double s = -tau + 2.0 * tau * j / J;
      int b[3];
      for (int k = 0; k < 3; ++k) b[k] = (int)floor((pw[k] + s * rw[k]) / voxel / kB);
      if (!key_in_range(b[0], b[1], b[2])) continue;
      uint64_t key = pack_key(b[0], b[1], b[2]);
      if (key == prev) continue;
      prev = key;
      insert_request(entries, req, mask, key, d, counters, max_entries);
    }
  }
}

// The frame's new brick requests, one entry per (block, direction) still without a brick:
// sort key (block key << 3 | D) and the block's hash slot, appended in thread order (the
// sort that follows fixes the order).  counters[14] counts them, also past `cap` (then the
// host grows the buffers and collects again).
__global__ __launch_bounds__(256) void collect_k(const HashEntry* __restrict__ entries,
                                                 uint32_t* req, uint32_t buckets,
                                                 uint64_t* keys, uint32_t* vals, int64_t cap,
                                                 int32_t* counters) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= buckets) return;
  const uint32_t r = req[s];
  if (!r) return;
  for (int d = 0; d < 6; ++d) {
    if (!((r >> d) & 1u) || entries[s].brick[d] >= 0) continue;
    const int i = atomicAdd(&counters[14], 1);
    if (i < cap) {
      keys[i] = (entries[s].key << 3) | (uint64_t)d;
      vals[i] = s;
    }
  }
}

// Pool index of the i-th request in (block key, D) order: the free list of recycled bricks
// first (ascending, popped from its end: counters[10] entries), then the unused end of the
// pool (counters[0]); beyond the capacity the request is dropped.  Counters are read here
// and updated by assign_counts_k afterwards.
__global__ __launch_bounds__(256) void assign_sorted_k(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals, int n,
                                                       HashEntry* entries, int4* bkey,
                                                       const int32_t* __restrict__ free_list,
                                                       uint32_t capacity,
                                                       const int32_t* __restrict__ counters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int free_n = max(counters[10], 0);
  int idx;
  if (i < free_n) {
    idx = free_list[free_n - 1 - i];
  } else {
    const int64_t j = (int64_t)counters[0] + (i - free_n);
    idx = j < (int64_t)capacity ? (int)j : -1;
  }
  if (idx < 0) return;
  const uint64_t kd = keys[i];
  const int d = (int)(kd & 7u);
  int bx, by, bz;
  unpack_key(kd >> 3, bx, by, bz);
  entries[vals[i]].brick[d] = idx;
  bkey[idx] = make_int4(bx, by, bz, d);
}

__global__ __launch_bounds__(256) void clear_req_k(uint32_t* req, uint32_t buckets) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < buckets) req[s] = 0;
}

__global__ void zero_counter_k(int32_t* c) {
  if (threadIdx.x == 0) *c = 0;
}

__global__ void assign_counts_k(int n, uint32_t capacity, int32_t* counters) {
  if (threadIdx.x != 0) return;
  const int free_n = max(counters[10], 0);
  const int popped = min(free_n, n);
  counters[10] = free_n - popped;
  const int rest = n - popped;
  const int room = max(0, (int)capacity - counters[0]);
  const int taken = min(rest, room);
  counters[0] += taken;
  counters[1] += rest - taken;
  counters[14] = 0;
}

// The carving guard of Sec. 3 per pixel: carving through pixel p is allowed unless a valid
// depth within a radius of two pixels differs from p's by more than tau.  It depends on the
// pixel only, so it is taken once per pixel instead of once per carved voxel.
__global__ __launch_bounds__(256) void carve_guard_k(const float* __restrict__ depth, Intr in,
                                                     double scale, double tau, int enabled,
                                                     uint8_t* __restrict__ ok_out) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  int v = blockIdx.y * blockDim.y + threadIdx.y;
  if (u >= in.W || v >= in.H) return;
  const double z = (double)depth[(size_t)v * in.W + u] * scale;
  bool ok = enabled != 0;
  for (int dv = -2; dv <= 2 && ok; ++dv)
    for (int du = -2; du <= 2; ++du) {
      int uu = u + du, vv = v + dv;
      if (uu < 0 || vv < 0 || uu >= in.W || vv >= in.H) continue;
      double z1 = (double)depth[(size_t)vv * in.W + uu] * scale;
      if (!(z1 > 0.0)) continue;
      if (fabs(z1 - z) > tau) {
        ok = false;
        break;
      }
    }
  ok_out[(size_t)v * in.W + u] = ok ? 1 : 0;
}

struct FuseArgs {
  const float* depth;
  const uint8_t* rgb;
  const float* nmap;
  const uint8_t* carve_ok;
  Intr in;
  double scale;
  Pose T;
  int2* counts;    // per listed brick: updated distances / colours, or null
};

__global__ void vis_reset_k(int32_t* counters) {
  if (threadIdx.x == 0) counters[11] = 0;
}

// Sums the per-brick update counts of the frame into counters[12] (distances) and
// counters[13] (colours); one workgroup.
__global__ __launch_bounds__(1024) void fuse_count_k(const int2* __restrict__ counts,
                                                     int32_t* counters) {
  __shared__ int sg[16], sc[16];
  const int n = counters[11];
  int g = 0, c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    g += counts[i].x;
    c += counts[i].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    g += __shfl_xor(g, o);
    c += __shfl_xor(c, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sg[threadIdx.x >> 6] = g;
    sc[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tg = 0, tc = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      tg += sg[w];
      tc += sc[w];
    }
    counters[12] = tg;
    counters[13] = tc;
  }
}

// Conservative frustum test of every brick in the pool, one thread per brick: a brick is
// listed unless all its voxel centres provably project outside the image or lie behind the
// camera (the centres lie in the box of its eight corner centres, whose projection bounds
// theirs when every corner is in front of the camera).  Fusion then visits the listed
// bricks only; a brick left out would have had no voxel updated.
__global__ __launch_bounds__(256) void cull_k(const int4* __restrict__ bkey, int n, Pose T,
                                              Intr in, double voxel, int32_t* list,
                                              int32_t* counters) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const int4 key = bkey[b];
  if (key.w < 0) return;
  double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
  int front = 0;
  for (int c = 0; c < 8; ++c) {
    const double x[3] = {(double)(key.x * kB + ((c & 1) ? kB - 1 : 0)) * voxel,
                         (double)(key.y * kB + ((c & 2) ? kB - 1 : 0)) * voxel,
                         (double)(key.z * kB + ((c & 4) ? kB - 1 : 0)) * voxel};
    const double xr[3] = {x[0] - T.t[0], x[1] - T.t[1], x[2] - T.t[2]};
    double xc[3];
    for (int k = 0; k < 3; ++k)
      xc[k] = T.R[k] * xr[0] + T.R[3 + k] * xr[1] + T.R[6 + k] * xr[2];
    if (!(xc[2] > 0.0)) continue;
    ++front;
    const double uf = in.fx * xc[0] / xc[2] + in.cx, vf = in.fy * xc[1] / xc[2] + in.cy;
    umin = fmin(umin, uf);
    umax = fmax(umax, uf);
    vmin = fmin(vmin, vf);
    vmax = fmax(vmax, vf);
  }
  if (front == 0) return;                 // every voxel behind the camera
  if (front == 8) {
    // a voxel is used when floor(uf + 0.5) lies in [0, W), i.e. uf in [-0.5, W - 0.5)
    constexpr double kMargin = 1e-3;      // pixels, for rounding between the two evaluations
    if (umax < -0.5 - kMargin || vmax < -0.5 - kMargin || umin > in.W - 0.5 + kMargin ||
        vmin > in.H - 0.5 + kMargin)
      return;
  }
  list[atomicAdd(&counters[11], 1)] = b;
}

// Voxel-projection fusion (Sec. 3) of one brick per workgroup.  A brick with any updated
// voxel refreshes its sub-block minima (sdf over voxels with w > 0) for the render index.
// With a.counts the brick's numbers of updated distances and colours are stored at its
// list position (integration statistics).
template <int F>
__global__ __launch_bounds__(256) void fuse_k(MapView m, FuseArgs a, float* sub_min,
                                              uint64_t* brick_neg,
                                              const int32_t* __restrict__ list,
                                              const int32_t* __restrict__ counters) {
  if ((int)blockIdx.x >= counters[11]) return;   // the grid covers the whole pool
  const int b = __builtin_amdgcn_readfirstlane(list[blockIdx.x]);
  const int4 key = m.bkey[b];
  const int D = key.w;
  if (D < 0) {                            // a recycled brick on the free list
    if (a.counts && threadIdx.x == 0) a.counts[blockIdx.x] = make_int2(0, 0);
    return;
  }
  const size_t HW = (size_t)a.in.W * a.in.H;
  const double tau = (double)m.tau;
  bool upd = false;
  int n_geo = 0, n_col = 0;    // voxels of this thread updated (at most two each)
  for (int l = threadIdx.x; l < kVox; l += blockDim.x) {
    const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
    double x[3] = {(double)(key.x * kB + lx) * m.voxel, (double)(key.y * kB + ly) * m.voxel,
                   (double)(key.z * kB + lz) * m.voxel};
    double xr[3] = {x[0] - a.T.t[0], x[1] - a.T.t[1], x[2] - a.T.t[2]};
    double xc[3];
    for (int k = 0; k < 3; ++k)
      xc[k] = a.T.R[k] * xr[0] + a.T.R[3 + k] * xr[1] + a.T.R[6 + k] * xr[2];
    if (!(xc[2] > 0.0)) continue;
    double uf = a.in.fx * xc[0] / xc[2] + a.in.cx;
    double vf = a.in.fy * xc[1] / xc[2] + a.in.cy;
    double ur = floor(uf + 0.5), vr = floor(vf + 0.5);
    if (ur < 0.0 || vr < 0.0 || ur >= (double)a.in.W || vr >= (double)a.in.H) continue;
    const int u = (int)ur, v = (int)vr;
    const size_t pi = (size_t)v * a.in.W + u;
    const float nx = a.nmap[pi], ny = a.nmap[HW + pi], nz = a.nmap[2 * HW + pi];
    if (nx == 0.f && ny == 0.f && nz == 0.f) continue;
    const double z = (double)a.depth[pi] * a.scale;
    if (!(z > 0.0) || !isfinite(z)) continue;
    const double pc[3] = {z * ((double)u - a.in.cx) / a.in.fx, z * ((double)v - a.in.cy) / a.in.fy, z};
    // point-to-plane distance (eq. point-to-plane) with the normal facing the camera, so that
    // positive values lie in front of the surface
    const double dd = ((xc[0] - pc[0]) * nx + (xc[1] - pc[1]) * ny + (xc[2] - pc[2]) * nz) / tau;
    const size_t vi = (size_t)b * kVox + l;
    if (dd > 1.0) {
      // free space: value 1 with a constant weight unless a depth jump above tau lies within
      // two pixels (Sec. 3; carve_guard_k)
      if (a.carve_ok[pi]) {
        float sd, w;
        Vox<F>::load(m.geo, vi, sd, w);
        const float nw = w + m.w_carve;
        Vox<F>::store(m.geo, vi, (sd * w + 1.0f * m.w_carve) / nw, fminf(nw, m.w_max));
        upd = true;
        ++n_geo;
      }
      continue;
    }
    if (dd < -1.0) continue;
    float nwx = (float)(a.T.R[0] * nx + a.T.R[1] * ny + a.T.R[2] * nz);
    float nwy = (float)(a.T.R[3] * nx + a.T.R[4] * ny + a.T.R[5] * nz);
    float nwz = (float)(a.T.R[6] * nx + a.T.R[7] * ny + a.T.R[8] * nz);
    const float wdir = w_dir_cos(axis_dot(nwx, nwy, nwz, D), m.theta);
    if (!(wdir > 0.f)) continue;
    // w_d = w_depth * w_angle * w_dir (eq. combined_fusion_weight), w_depth = 1,
    // w_angle = max(0, <n, -r>) for the unit ray r through the pixel
    const double plen = sqrt(pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
    const float w_angle = fmaxf(0.f, (float)(-(pc[0] * nx + pc[1] * ny + pc[2] * nz) / plen));
    const float wd = w_angle * wdir;
    if (wd < m.w_min) continue;
    {
      float sd, w;
      Vox<F>::load(m.geo, vi, sd, w);
      const float nw = w + wd;
      Vox<F>::store(m.geo, vi, (sd * w + (float)dd * wd) / nw, fminf(nw, m.w_max));
    }
    upd = true;
    ++n_geo;
    if (m.with_color && a.rgb) {
      // colour weight w_c = w_d (1 - min(1, |p - x| / tau)) (eq. color_weight)
      const double dist = sqrt((pc[0] - xc[0]) * (pc[0] - xc[0]) + (pc[1] - xc[1]) * (pc[1] - xc[1]) +
                               (pc[2] - xc[2]) * (pc[2] - xc[2]));
      const float wc = wd * (1.0f - fminf(1.0f, (float)(dist / tau)));
      if (wc > 0.f) {
        float Wc;
        uint32_t c;
        Vox<F>::load_color(m.rgb, m.wc, vi, c, Wc);
        const float inv = 1.0f / (Wc + wc);
        uint32_t outc = 0;
        for (int ch = 0; ch < 3; ++ch) {
          float old = (float)((c >> (8 * ch)) & 0xFFu);
          float px = (float)a.rgb[3 * pi + ch];
          float val = rintf((old * Wc + px * wc) * inv);
          val = fminf(255.f, fmaxf(0.f, val));
          outc |= (uint32_t)val << (8 * ch);
        }
        Vox<F>::store_color(m.rgb, m.wc, vi, outc, fminf(Wc + wc, m.w_max));
        ++n_col;
      }
    }
  }
  if (a.counts) {
    // both counts packed in one word (at most 512 each): wave sums, then the workgroup's
    __shared__ int wsum[4];
    int cnt = n_geo | (n_col << 16);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
      a.counts[blockIdx.x] = make_int2(t & 0xFFFF, t >> 16);
    }
  }
  if (__syncthreads_or(upd))
    brick_sub_min<F>(m.geo, b, sub_min + (size_t)b * 8, brick_neg + (size_t)b * 16);
}

Intr make_intr(const dtsdf_intrinsics* i) {
  return Intr{i->width, i->height, (double)i->fx, (double)i->fy, (double)i->cx, (double)i->cy};
}

Pose make_pose(const double T[16]) {
  Pose p;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) p.R[3 * r + c] = T[4 * r + c];
    p.t[r] = T[4 * r + 3];
  }
  return p;
}

bool valid_intr(const dtsdf_intrinsics* i) {
  return i && i->width > 2 && i->height > 2 && i->width <= 16384 && i->height <= 16384 &&
         i->fx > 0 && i->fy > 0;
}

}  // namespace

namespace {

// The bricks-handed-out counter may overshoot the pool while a frame allocates; it is
// brought back to the capacity on the device (no host word travels to the device).
__global__ void clamp_handed_k(int32_t* counters, int32_t cap) {
  if (threadIdx.x == 0 && counters[0] > cap) counters[0] = cap;
}

}  // namespace

namespace dtsdf {

void launch_clamp_handed(dtsdf_map* m, hipStream_t st) {
  hipLaunchKernelGGL(clamp_handed_k, dim3(1), dim3(64), 0, st, m->counters,
                     (int32_t)m->p.brick_capacity);
}

// Every caller runs launch_bbox next, which clamps the free-list count.
namespace {
// Grows the request buffers to `n` entries and the sort scratch to what sorting them needs.
dtsdf_status ensure_alloc_buffers(dtsdf_map* m, int64_t n, hipStream_t st) {
  if (n > m->alloc_cap) {
    DTSDF_HIP(hipStreamSynchronize(st));
    (void)hipFree(m->alloc_keys);
    (void)hipFree(m->alloc_vals);
    m->alloc_keys = nullptr;
    m->alloc_vals = nullptr;
    m->alloc_cap = 0;
    const int64_t cap = std::max<int64_t>(n, 1 << 16) * 5 / 4;
    if (hipMalloc(&m->alloc_keys, sizeof(uint64_t) * 2 * cap) != hipSuccess ||
        hipMalloc(&m->alloc_vals, sizeof(uint32_t) * 2 * cap) != hipSuccess)
      return DTSDF_E_NOMEM;
    m->alloc_cap = cap;
  }
  size_t need = 0;
  DTSDF_HIP(hipcub::DeviceRadixSort::SortPairs(
      nullptr, need, m->alloc_keys, m->alloc_keys + m->alloc_cap, m->alloc_vals,
      m->alloc_vals + m->alloc_cap, (int)m->alloc_cap, 0, 63, st));
  size_t need_free = 0;
  DTSDF_HIP(hipcub::DeviceRadixSort::SortKeys(
      nullptr, need_free, m->free_list, m->free_list, (int)m->p.brick_capacity, 0, 32, st));
  need = std::max(need, need_free);
  if (need > m->sort_tmp_bytes) {
    DTSDF_HIP(hipStreamSynchronize(st));
    (void)hipFree(m->sort_tmp);
    m->sort_tmp = nullptr;
    m->sort_tmp_bytes = 0;
    if (hipMalloc(&m->sort_tmp, need) != hipSuccess) return DTSDF_E_NOMEM;
    m->sort_tmp_bytes = need;
  }
  return DTSDF_OK;
}
}  // namespace

dtsdf_status launch_assign(dtsdf_map* m, hipStream_t st) {
  if (m->alloc_cap == 0) {
    const dtsdf_status s0 = ensure_alloc_buffers(m, 1 << 16, st);
    if (s0 != DTSDF_OK) return s0;
  }
  const dim3 gb((m->buckets + 255) / 256);
  int32_t n = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    hipLaunchKernelGGL(zero_counter_k, dim3(1), dim3(64), 0, st, m->counters + 14);
    hipLaunchKernelGGL(collect_k, gb, dim3(256), 0, st, m->entries, m->req, m->buckets,
                       m->alloc_keys, m->alloc_vals, m->alloc_cap, m->counters);
    DTSDF_HIP(hipMemcpyAsync(&n, m->counters + 14, sizeof(n), hipMemcpyDeviceToHost, st));
    DTSDF_HIP(hipStreamSynchronize(st));
    if (n <= m->alloc_cap) break;
    // more requests than the buffers hold: grow them and collect again (the request bits
    // are still set)
    const dtsdf_status sg = ensure_alloc_buffers(m, n, st);
    if (sg != DTSDF_OK) return sg;
  }
  if (n > m->alloc_cap) return DTSDF_E_NOMEM;
  hipLaunchKernelGGL(clear_req_k, gb, dim3(256), 0, st, m->req, m->buckets);
  if (n > 0) {
    uint64_t* k_in = m->alloc_keys;
    uint64_t* k_out = m->alloc_keys + m->alloc_cap;
    uint32_t* v_in = m->alloc_vals;
    uint32_t* v_out = m->alloc_vals + m->alloc_cap;
    size_t bytes = m->sort_tmp_bytes;
    DTSDF_HIP(hipcub::DeviceRadixSort::SortPairs(m->sort_tmp, bytes, k_in, k_out, v_in, v_out,
                                                 n, 0, 63, st));
    hipLaunchKernelGGL(assign_sorted_k, dim3((n + 255) / 256), dim3(256), 0, st, k_out, v_out,
                       n, m->entries, m->bkey, m->free_list, m->p.brick_capacity,
                       m->counters);
  }
  hipLaunchKernelGGL(assign_counts_k, dim3(1), dim3(64), 0, st, n, m->p.brick_capacity,
                     m->counters);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

dtsdf_status sort_free_list(dtsdf_map* m, hipStream_t st) {
  if (m->n_free <= 1) return DTSDF_OK;
  // sorted into the request key buffer (grown to hold the list) and copied back
  const dtsdf_status s0 = ensure_alloc_buffers(m, std::max<int64_t>(m->n_free / 2 + 1, 1 << 16), st);
  if (s0 != DTSDF_OK) return s0;
  int32_t* tmp = reinterpret_cast<int32_t*>(m->alloc_keys);
  size_t bytes = m->sort_tmp_bytes;
  DTSDF_HIP(hipcub::DeviceRadixSort::SortKeys(m->sort_tmp, bytes, m->free_list, tmp,
                                              (int)m->n_free, 0, 32, st));
  DTSDF_HIP(hipMemcpyAsync(m->free_list, tmp, sizeof(int32_t) * m->n_free,
                           hipMemcpyDeviceToDevice, st));
  return DTSDF_OK;
}

}  // namespace dtsdf

extern "C" {

dtsdf_status dtsdf_vertex_normal(const float* depth, const dtsdf_intrinsics* intr,
                                 float depth_scale, float* vertex, float* normal,
                                 void* stream) {
  if (!depth || !vertex || !normal || !valid_intr(intr) || !(depth_scale > 0))
    return DTSDF_E_INVAL;
  Intr in = make_intr(intr);
  dim3 blk(16, 16), grd((in.W + 15) / 16, (in.H + 15) / 16);
  hipLaunchKernelGGL(vertex_normal_k, grd, blk, 0, (hipStream_t)stream, depth, in,
                     (double)depth_scale, vertex, normal);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

dtsdf_status dtsdf_depth_downsample(const float* depth_in, int32_t width, int32_t height,
                                    float* depth_out, void* stream) {
  if (!depth_in || !depth_out || width < 2 || height < 2) return DTSDF_E_INVAL;
  dim3 blk(16, 16), grd((width / 2 + 15) / 16, (height / 2 + 15) / 16);
  hipLaunchKernelGGL(downsample_k, grd, blk, 0, (hipStream_t)stream, depth_in, width, height,
                     depth_out);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

}  // extern "C"

namespace {

// Fusion of one frame; `normal` (device, planar 3 x H x W, camera frame) replaces the
// cross-product normals when given.
dtsdf_status integrate_impl(dtsdf_map* m, const float* depth, const float* normal,
                            const uint8_t* rgb, const dtsdf_intrinsics* intr,
                            const double T_world_cam[16], float depth_scale, void* stream,
                            dtsdf_integrate_stats* stats) {
  if (!m || m->regular || !depth || !valid_intr(intr) || !T_world_cam || !(depth_scale > 0))
    return DTSDF_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  Intr in = make_intr(intr);
  const int64_t HW = (int64_t)in.W * in.H;
  if (!normal && HW > m->img_cap) {
    DTSDF_HIP(hipStreamSynchronize(st));
    (void)hipFree(m->vmap);
    (void)hipFree(m->nmap);
    m->vmap = m->nmap = nullptr;
    m->img_cap = 0;
    if (hipMalloc(&m->vmap, sizeof(float) * 3 * HW) != hipSuccess ||
        hipMalloc(&m->nmap, sizeof(float) * 3 * HW) != hipSuccess)
      return DTSDF_E_NOMEM;
    m->img_cap = HW;
  }
  Pose T = make_pose(T_world_cam);
  dim3 blk(16, 16), grd((in.W + 15) / 16, (in.H + 15) / 16);
  if (!normal)
    hipLaunchKernelGGL(vertex_normal_k, grd, blk, 0, st, depth, in, (double)depth_scale,
                       m->vmap, m->nmap);
  const float* nmap = normal ? normal : m->nmap;
  const int64_t before = m->n_bricks - m->n_free;
  int64_t dropped_now = 0;
  if (!m->p.dense) {
    const double voxel = (double)m->p.voxel_size, tau = (double)m->p.truncation;
    const int J = (int)std::ceil(2.0 * tau / voxel - 1e-9);
    const int32_t max_entries = (int32_t)((uint64_t)m->buckets * 3 / 4);
    hipLaunchKernelGGL(request_k, grd, blk, 0, st, depth, nmap, in, (double)depth_scale, T,
                       voxel, tau, J, m->p.theta, m->entries, m->req, m->buckets - 1,
                       m->counters, max_entries);
    const dtsdf_status as = launch_assign(m, st);
    if (as != DTSDF_OK) return as;
    launch_bbox(m, st);
    int32_t c[11];
    DTSDF_HIP(hipMemcpyAsync(c, m->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    DTSDF_HIP(hipStreamSynchronize(st));
    dtsdf_status gs = ensure_grid(m, c + 4, st);
    if (gs != DTSDF_OK) return gs;
    int64_t handed = c[0];
    if (handed > (int64_t)m->p.brick_capacity) {
      launch_clamp_handed(m, st);
      handed = m->p.brick_capacity;
    }
    dropped_now = (int64_t)c[1] - m->dropped;
    m->dropped = c[1];
    m->n_bricks = handed;
    m->n_blocks = c[3];
    m->n_free = c[10];
  }
  if (m->n_bricks > 0 && HW > m->carve_cap) {
    DTSDF_HIP(hipStreamSynchronize(st));
    (void)hipFree(m->carve_ok);
    m->carve_ok = nullptr;
    m->carve_cap = 0;
    if (hipMalloc(&m->carve_ok, (size_t)HW) != hipSuccess) return DTSDF_E_NOMEM;
    m->carve_cap = HW;
  }
  if (m->n_bricks > 0) {
    hipLaunchKernelGGL(carve_guard_k, grd, blk, 0, st, depth, in, (double)depth_scale,
                       (double)m->p.truncation, m->p.w_carve > 0.f ? 1 : 0, m->carve_ok);
    // the visible-brick count starts at zero: cleared by the bounding-box reset of the
    // sparse path above, here for dense maps
    if (m->p.dense) hipLaunchKernelGGL(vis_reset_k, dim3(1), dim3(64), 0, st, m->counters);
    const int n = (int)m->n_bricks;
    hipLaunchKernelGGL(cull_k, dim3((n + 255) / 256), dim3(256), 0, st, m->bkey, n, T, in,
                       (double)m->p.voxel_size, m->vis_list, m->counters);
    if (stats && !m->fuse_cnt &&
        hipMalloc(&m->fuse_cnt, sizeof(int2) * (size_t)m->p.brick_capacity) != hipSuccess) {
      m->fuse_cnt = nullptr;
      return DTSDF_E_NOMEM;
    }
    FuseArgs fa{depth, rgb, nmap, m->carve_ok, in, (double)depth_scale, T,
                stats ? m->fuse_cnt : nullptr};
    const dim3 grd_b((uint32_t)n);
    if (m->fmt == 0)
      hipLaunchKernelGGL(fuse_k<0>, grd_b, dim3(256), 0, st, make_view(m), fa, m->sub_min,
                         m->brick_neg, m->vis_list, m->counters);
    else if (m->fmt == 1)
      hipLaunchKernelGGL(fuse_k<1>, grd_b, dim3(256), 0, st, make_view(m), fa, m->sub_min,
                         m->brick_neg, m->vis_list, m->counters);
    else
      hipLaunchKernelGGL(fuse_k<2>, grd_b, dim3(256), 0, st, make_view(m), fa, m->sub_min,
                         m->brick_neg, m->vis_list, m->counters);
  }
  if (stats && m->n_bricks > 0)
    hipLaunchKernelGGL(fuse_count_k, dim3(1), dim3(1024), 0, st, m->fuse_cnt, m->counters);
  DTSDF_HIP(hipGetLastError());
  dtsdf_status is = launch_index_update(m, st);
  if (is != DTSDF_OK) return is;
  if (stats) {
    stats->new_bricks = m->n_bricks - m->n_free - before;
    stats->dropped = dropped_now;
    stats->bricks = m->n_bricks - m->n_free;
    int32_t fc[3] = {0, 0, 0};
    if (m->n_bricks > 0)
      DTSDF_HIP(hipMemcpyAsync(fc, m->counters + 11, sizeof(fc), hipMemcpyDeviceToHost, st));
    DTSDF_HIP(hipStreamSynchronize(st));
    stats->visited_bricks = fc[0];
    stats->updated_voxels = fc[1];
    stats->color_voxels = fc[2];
  }
  return dropped_now > 0 ? DTSDF_E_CAPACITY : DTSDF_OK;
}

}  // namespace

extern "C" {

dtsdf_status dtsdf_integrate(dtsdf_map* m, const float* depth, const uint8_t* rgb,
                             const dtsdf_intrinsics* intr, const double T_world_cam[16],
                             float depth_scale, void* stream, dtsdf_integrate_stats* stats) {
  return integrate_impl(m, depth, nullptr, rgb, intr, T_world_cam, depth_scale, stream, stats);
}

dtsdf_status dtsdf_integrate_normals(dtsdf_map* m, const float* depth, const float* normal,
                                     const uint8_t* rgb, const dtsdf_intrinsics* intr,
                                     const double T_world_cam[16], float depth_scale,
                                     void* stream, dtsdf_integrate_stats* stats) {
  if (!normal) return DTSDF_E_INVAL;
  return integrate_impl(m, depth, normal, rgb, intr, T_world_cam, depth_scale, stream, stats);
}

}  // extern "C"
