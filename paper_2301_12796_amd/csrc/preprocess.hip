// Input preprocessing (Sec. 7; parameters of Sec. 8) and the post-fusion error (Sec. 8).
//
//   depth_filter_k   one workgroup per 16x16 output tile: the raw depth of the tile plus a
//                    (radius + 1) halo is staged in LDS, the support filter (a pixel keeps its
//                    depth only with >= min_support of its eight neighbours within
//                    support_rel * D(p)) is evaluated on the tile plus a radius halo into a
//                    second LDS tile, and the bilateral filter reads that tile.  The support
//                    tests are exact (float64 on float32 inputs); the bilateral sums are
//                    float32, accumulated relative to the centre depth.
//   normal_filter_k  one workgroup per 16x16 tile of a planar (3, H, W) normal map with a
//                    radius halo in LDS; range weight from the angle between normals in
//                    degrees, taken as atan2(|n x q|, n . q), which stays accurate for nearly
//                    parallel normals.
//   depth_error_k    one workgroup of 1024 threads, fixed-order float64 sums of |a - b| and
//                    of the count over pixels where both depths are valid: deterministic.
#include <cmath>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

constexpr int kTile = 16;
constexpr int kMaxRadius = 8;
constexpr int kRawSide = kTile + 2 * (kMaxRadius + 1);    // 34
constexpr int kSupSide = kTile + 2 * kMaxRadius;          // 32
constexpr int kWin = 2 * kMaxRadius + 1;                  // 17

struct DepthFilterArgs {
  const float* in;
  float* out;
  int W, H;
  float support_rel;
  int min_support;
  float inv2sd2, inv2sr2;
  int R;
};

__global__ __launch_bounds__(256) void depth_filter_k(DepthFilterArgs a) {
  __shared__ float raw[kRawSide * kRawSide];
  __shared__ float sup[kSupSide * kSupSide];
  __shared__ float ws[kWin * kWin];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const int R = a.R, rs = kTile + 2 * (R + 1), ss = kTile + 2 * R, win = 2 * R + 1;
  for (int i = tid; i < rs * rs; i += 256) {
    const int x = x0 - R - 1 + i % rs, y = y0 - R - 1 + i / rs;
    raw[i] = (x >= 0 && y >= 0 && x < a.W && y < a.H) ? a.in[(size_t)y * a.W + x] : 0.f;
  }
  for (int i = tid; i < win * win; i += 256) {
    const int du = i % win - R, dv = i / win - R;
    ws[i] = __expf(-(float)(du * du + dv * dv) * a.inv2sd2);
  }
  __syncthreads();
  for (int i = tid; i < ss * ss; i += 256) {
    const int sx = i % ss, sy = i / ss;         // raw index (sx + 1, sy + 1)
    const float d = raw[(sy + 1) * rs + sx + 1];
    float keep = 0.f;
    if (d > 0.f) {
      if (a.min_support <= 0) {
        keep = d;
      } else {
        const double lim = (double)a.support_rel * (double)d;
        int cnt = 0;
        for (int dv = -1; dv <= 1; ++dv)
          for (int du = -1; du <= 1; ++du) {
            if (du == 0 && dv == 0) continue;
            const float q = raw[(sy + 1 + dv) * rs + sx + 1 + du];
            cnt += (q > 0.f && fabs((double)q - (double)d) <= lim) ? 1 : 0;
          }
        keep = cnt >= a.min_support ? d : 0.f;
      }
    }
    sup[i] = keep;
  }
  __syncthreads();
  const int tx = tid % kTile, ty = tid / kTile;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= a.W || y >= a.H) return;
  const float d = sup[(ty + R) * ss + tx + R];
  float res = 0.f;
  if (d > 0.f) {
    float num = 0.f, den = 0.f;
    for (int dv = 0; dv < win; ++dv) {
      const float* row = sup + (ty + dv) * ss + tx;
      const float* wrow = ws + dv * win;
      for (int du = 0; du < win; ++du) {
        const float q = row[du];
        if (q > 0.f) {
          const float e = q - d;
          const float w = wrow[du] * __expf(-e * e * a.inv2sr2);
          num += w * e;
          den += w;
        }
      }
    }
    res = d + num / den;
  }
  a.out[(size_t)y * a.W + x] = res;
}

struct NormalFilterArgs {
  const float* in;
  float* out;
  int W, H;
  float inv2sd2, inv2sr2;      // inv2sr2 in 1 / deg^2
  int R;
};

__global__ __launch_bounds__(256) void normal_filter_k(NormalFilterArgs a) {
  __shared__ float nx[kSupSide * kSupSide], ny[kSupSide * kSupSide], nz[kSupSide * kSupSide];
  __shared__ float ws[kWin * kWin];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const int R = a.R, ss = kTile + 2 * R, win = 2 * R + 1;
  const size_t HW = (size_t)a.W * a.H;
  for (int i = tid; i < ss * ss; i += 256) {
    const int x = x0 - R + i % ss, y = y0 - R + i / ss;
    const bool in = x >= 0 && y >= 0 && x < a.W && y < a.H;
    const size_t p = in ? (size_t)y * a.W + x : 0;
    nx[i] = in ? a.in[p] : 0.f;
    ny[i] = in ? a.in[HW + p] : 0.f;
    nz[i] = in ? a.in[2 * HW + p] : 0.f;
  }
  for (int i = tid; i < win * win; i += 256) {
    const int du = i % win - R, dv = i / win - R;
    ws[i] = __expf(-(float)(du * du + dv * dv) * a.inv2sd2);
  }
  __syncthreads();
  const int tx = tid % kTile, ty = tid / kTile;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= a.W || y >= a.H) return;
  const int c = (ty + R) * ss + tx + R;
  const float px = nx[c], py = ny[c], pz = nz[c];
  float o[3] = {0.f, 0.f, 0.f};
  if (px != 0.f || py != 0.f || pz != 0.f) {
    constexpr float kDeg = 57.29577951308232f;
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int dv = 0; dv < win; ++dv)
      for (int du = 0; du < win; ++du) {
        const int j = (ty + dv) * ss + tx + du;
        const float qx = nx[j], qy = ny[j], qz = nz[j];
        if (qx == 0.f && qy == 0.f && qz == 0.f) continue;
        const float cx = py * qz - pz * qy, cy = pz * qx - px * qz, cz = px * qy - py * qx;
        const float ang = atan2f(sqrtf(cx * cx + cy * cy + cz * cz), px * qx + py * qy + pz * qz) * kDeg;
        const float w = ws[dv * win + du] * __expf(-ang * ang * a.inv2sr2);
        ax += w * qx;
        ay += w * qy;
        az += w * qz;
      }
    const float ln = sqrtf(ax * ax + ay * ay + az * az);
    if (ln > 0.f) {
      o[0] = ax / ln;
      o[1] = ay / ln;
      o[2] = az / ln;
    }
  }
  const size_t p = (size_t)y * a.W + x;
  a.out[p] = o[0];
  a.out[HW + p] = o[1];
  a.out[2 * HW + p] = o[2];
}

__device__ inline void err_acc(float a, float b, double& s, double& c) {
  if (a > 0.f && b > 0.f) {
    s += fabs((double)a - (double)b);
    c += 1.0;
  }
}

// vec: both images 16-byte aligned; the first n4 = n / 4 groups of four pixels are read as
// float4 (four groups per thread and pass, so that enough loads are in flight for one
// workgroup), the tail pixel by pixel.  The assignment of pixels to threads is fixed.
__global__ __launch_bounds__(1024) void depth_error_k(const float* __restrict__ r,
                                                      const float* __restrict__ m, size_t n,
                                                      int vec, double* out) {
  __shared__ double ss[1024], sc[1024];
  double s = 0.0, c = 0.0;
  size_t done = 0;
  if (vec) {
    const size_t n4 = n / 4;
    const float4* r4 = reinterpret_cast<const float4*>(r);
    const float4* m4 = reinterpret_cast<const float4*>(m);
    for (size_t base = 0; base < n4; base += 4 * 1024) {
      float4 a[4], b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t i = base + k * 1024 + threadIdx.x;
        a[k] = i < n4 ? r4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        b[k] = i < n4 ? m4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        err_acc(a[k].x, b[k].x, s, c);
        err_acc(a[k].y, b[k].y, s, c);
        err_acc(a[k].z, b[k].z, s, c);
        err_acc(a[k].w, b[k].w, s, c);
      }
    }
    done = n4 * 4;
  }
  for (size_t i = done + threadIdx.x; i < n; i += 1024) err_acc(r[i], m[i], s, c);
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sc[threadIdx.x] += sc[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ss[0];
    out[1] = sc[0];
  }
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

}  // namespace

extern "C" {

dtsdf_status dtsdf_depth_filter(const float* depth_in, int32_t width, int32_t height,
                                const dtsdf_depth_filter_params* p, float* depth_out,
                                void* stream) {
  if (!depth_in || !depth_out || depth_in == depth_out || !p || width <= 0 || height <= 0 ||
      p->radius < 0 || p->radius > kMaxRadius || p->min_support > 8 ||
      !(p->support_rel >= 0.f) || (p->radius > 0 && (!finite_pos(p->sigma_d) ||
                                                    !finite_pos(p->sigma_r))))
    return DTSDF_E_INVAL;
  DepthFilterArgs a;
  a.in = depth_in;
  a.out = depth_out;
  a.W = width;
  a.H = height;
  a.support_rel = p->support_rel;
  a.min_support = p->min_support;
  a.R = p->radius;
  a.inv2sd2 = p->radius > 0 ? 1.f / (2.f * p->sigma_d * p->sigma_d) : 0.f;
  a.inv2sr2 = p->radius > 0 ? 1.f / (2.f * p->sigma_r * p->sigma_r) : 0.f;
  dim3 grd((width + kTile - 1) / kTile, (height + kTile - 1) / kTile);
  hipLaunchKernelGGL(depth_filter_k, grd, dim3(256), 0, (hipStream_t)stream, a);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

dtsdf_status dtsdf_normal_filter(const float* normal_in, int32_t width, int32_t height,
                                 float sigma_d, float sigma_r_deg, int32_t radius,
                                 float* normal_out, void* stream) {
  if (!normal_in || !normal_out || normal_in == normal_out || width <= 0 || height <= 0 ||
      radius < 0 || radius > kMaxRadius || !finite_pos(sigma_d) || !finite_pos(sigma_r_deg))
    return DTSDF_E_INVAL;
  NormalFilterArgs a;
  a.in = normal_in;
  a.out = normal_out;
  a.W = width;
  a.H = height;
  a.R = radius;
  a.inv2sd2 = 1.f / (2.f * sigma_d * sigma_d);
  a.inv2sr2 = 1.f / (2.f * sigma_r_deg * sigma_r_deg);
  dim3 grd((width + kTile - 1) / kTile, (height + kTile - 1) / kTile);
  hipLaunchKernelGGL(normal_filter_k, grd, dim3(256), 0, (hipStream_t)stream, a);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

dtsdf_status dtsdf_depth_error(const float* rendered, const float* measured, int32_t width,
                               int32_t height, double* out, void* stream) {
  if (!rendered || !measured || !out || width <= 0 || height <= 0) return DTSDF_E_INVAL;
  const int vec = (((uintptr_t)rendered | (uintptr_t)measured) & 15u) == 0 ? 1 : 0;
  hipLaunchKernelGGL(depth_error_k, dim3(1), dim3(1024), 0, (hipStream_t)stream, rendered,
                     measured, (size_t)width * height, vec, out);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

}  // extern "C"
