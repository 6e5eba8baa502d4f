// Point-to-plane ICP step in SE(3) and Sim(3) (Sec. 5 and Sec. 6).
//
//   reduce_k<DIM>  per live pixel: transform, projective association, rejection, residual
//                  r = <q - y, n> and Jacobian J = (-n, -(y x n)[, -<n, y>]); every thread
//                  sums a fixed strided subset of pixels in float32, the workgroup folds its
//                  four waves with xor shuffles and a fixed-order LDS pass, and writes one
//                  partial vector.  No atomics: the result is bitwise reproducible (the paper
//                  replaced atomic block sums for exactly this reason, Sec. 5).
//   solve_k<DIM>   one workgroup: float64 sum of the partials in block order, Cholesky
//                  factorisation of H (eq. ICP_Hessian; the factor 2 cancels), xi = -H^-1 g
//                  (eq. ICP_solution), exp(xi) in closed form and T <- exp(xi) T
//                  (eq. deltaT_update), all on the device.
#include <mutex>
#include <vector>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

constexpr int kReduceBlocks = 512;
constexpr int kReduceThreads = 256;

template <int DIM>
struct Sizes {
  static constexpr int NH = DIM * (DIM + 1) / 2;
  static constexpr int NS = NH + DIM + 2;   // H upper triangle, g, error, count
};

struct IcpArgs {
  const float* lv;
  const float* ln;
  int lW, lH;
  const float* mv;
  const float* mn;
  const uint8_t* mmask;
  int mW, mH;
  float fx, fy, cx, cy;   // model intrinsics
  float max_dist2, cos_angle;
  int weight_kind;
  float z_min;
  const double* pose;     // device 4x4 row-major, live -> model
};

struct ResultDev {
  double xi[7];
  double H[49];
  double g[7];
  double err;
  double count;
  double step;
  int status;     // 0 ok, 1 too few inliers, 2 not positive definite
  int pad;
};

template <int DIM>
__global__ __launch_bounds__(kReduceThreads) void reduce_k(IcpArgs a, float* partials) {
  constexpr int NS = Sizes<DIM>::NS;
  constexpr int NH = Sizes<DIM>::NH;
  float acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.f;
  float R[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R[3 * r + c] = (float)a.pose[4 * r + c];
    t[r] = (float)a.pose[4 * r + 3];
  }
  const size_t LHW = (size_t)a.lW * a.lH;
  const size_t MHW = (size_t)a.mW * a.mH;
  for (size_t i = (size_t)blockIdx.x * kReduceThreads + threadIdx.x; i < LHW;
       i += (size_t)gridDim.x * kReduceThreads) {
    const float nlx = a.ln[i], nly = a.ln[LHW + i], nlz = a.ln[2 * LHW + i];
    if (nlx == 0.f && nly == 0.f && nlz == 0.f) continue;
    const float px = a.lv[i], py = a.lv[LHW + i], pz = a.lv[2 * LHW + i];
    float y[3], nr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      y[k] = R[3 * k] * px + R[3 * k + 1] * py + R[3 * k + 2] * pz + t[k];
      nr[k] = R[3 * k] * nlx + R[3 * k + 1] * nly + R[3 * k + 2] * nlz;
    }
    if (!(y[2] > 0.f)) continue;
    const float inr = 1.f / sqrtf(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    const float uf = a.fx * y[0] / y[2] + a.cx;
    const float vf = a.fy * y[1] / y[2] + a.cy;
    const float ur = floorf(uf + 0.5f), vr = floorf(vf + 0.5f);
    if (!(ur >= 0.f && vr >= 0.f && ur < (float)a.mW && vr < (float)a.mH)) continue;
    const size_t mi = (size_t)vr * a.mW + (size_t)ur;
    if (a.mmask && !a.mmask[mi]) continue;
    const float n[3] = {a.mn[mi], a.mn[MHW + mi], a.mn[2 * MHW + mi]};
    if (!a.mmask && n[0] == 0.f && n[1] == 0.f && n[2] == 0.f) continue;
    const float d[3] = {a.mv[mi] - y[0], a.mv[MHW + mi] - y[1], a.mv[2 * MHW + mi] - y[2]};
    if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > a.max_dist2) continue;
    if ((n[0] * nr[0] + n[1] * nr[1] + n[2] * nr[2]) * inr < a.cos_angle) continue;
    const float res = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    float J[DIM];
    J[0] = -n[0];
    J[1] = -n[1];
    J[2] = -n[2];
    J[3] = -(y[1] * n[2] - y[2] * n[1]);
    J[4] = -(y[2] * n[0] - y[0] * n[2]);
    J[5] = -(y[0] * n[1] - y[1] * n[0]);
    if (DIM == 7) J[DIM - 1] = -(n[0] * y[0] + n[1] * y[1] + n[2] * y[2]);
    float w = 1.f;
    if (a.weight_kind == DTSDF_ICP_W_DEPTH) {
      const float zz = pz + (1.f - a.z_min);       // eq. ICP_weight
      w = 1.f / (zz * zz);
    }
    int s = 0;
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
      for (int c = r; c < DIM; ++c) acc[s++] += w * J[r] * J[c];
#pragma unroll
    for (int r = 0; r < DIM; ++r) acc[NH + r] += w * J[r] * res;
    acc[NS - 2] += w * res * res;
    acc[NS - 1] += 1.f;
  }
  __shared__ float lds[kReduceThreads / 64][NS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    float v = acc[s];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) lds[wave][s] = v;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    float v = 0.f;
    for (int wv = 0; wv < kReduceThreads / 64; ++wv) v += lds[wv][threadIdx.x];
    partials[(size_t)blockIdx.x * NS + threadIdx.x] = v;
  }
}

// exp of xi = (nu, omega[, sigma]) as a 4x4 row-major matrix (closed form).
__device__ void exp_sim3(const double* xi, int dim, double* E) {
  const double wx = xi[3], wy = xi[4], wz = xi[5];
  const double sg = dim == 7 ? xi[6] : 0.0;
  const double th2 = wx * wx + wy * wy + wz * wz;
  const double th = sqrt(th2);
  double W[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
  double W2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
  double A1, B1;       // rotation: I + A1 W + B1 W^2 (Rodrigues)
  if (th < 1e-4) {
    A1 = 1.0 - th2 / 6.0;
    B1 = 0.5 - th2 / 24.0;
  } else {
    A1 = sin(th) / th;
    B1 = (1.0 - cos(th)) / th2;
  }
  // V = int_0^1 e^(sigma u) exp(u W) du = a I + b W + c W^2
  const double es = exp(sg);
  double va, vb, vc;
  va = fabs(sg) < 1e-6 ? 1.0 + sg / 2.0 + sg * sg / 6.0 : (es - 1.0) / sg;
  if (th < 1e-3) {
    if (fabs(sg) < 1e-4) {
      vb = 0.5 + sg / 3.0 + sg * sg / 8.0 - th2 / 24.0;
      vc = 1.0 / 6.0 + sg / 8.0 + sg * sg / 20.0 - th2 / 120.0;
    } else {
      vb = (es * (sg - 1.0) + 1.0) / (sg * sg);
      vc = (es * (sg * sg - 2.0 * sg + 2.0) - 2.0) / (2.0 * sg * sg * sg);
    }
  } else if (fabs(sg) < 1e-12) {
    vb = (1.0 - cos(th)) / th2;
    vc = (th - sin(th)) / (th2 * th);
  } else {
    const double den = sg * sg + th2;
    vb = (es * (sg * sin(th) - th * cos(th)) + th) / (th * den);
    vc = (va - (es * (sg * cos(th) + th * sin(th)) - sg) / den) / th2;
  }
  for (int r = 0; r < 3; ++r) {
    double tr = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double I = r == c ? 1.0 : 0.0;
      E[4 * r + c] = es * (I + A1 * W[3 * r + c] + B1 * W2[3 * r + c]);
      tr += (va * I + vb * W[3 * r + c] + vc * W2[3 * r + c]) * xi[c];
    }
    E[4 * r + 3] = tr;
  }
  E[12] = E[13] = E[14] = 0.0;
  E[15] = 1.0;
}

template <int DIM>
__global__ __launch_bounds__(64) void solve_k(const float* partials, int nblocks,
                                             int min_inliers, double* pose, ResultDev* res) {
  constexpr int NS = Sizes<DIM>::NS;
  constexpr int NH = Sizes<DIM>::NH;
  __shared__ double sums[NS];
  if (threadIdx.x < NS) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += (double)partials[(size_t)b * NS + threadIdx.x];
    sums[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double H[DIM * DIM], g[DIM], L[DIM * DIM], y[DIM], xi[7] = {0, 0, 0, 0, 0, 0, 0};
  int s = 0;
  for (int r = 0; r < DIM; ++r)
    for (int c = r; c < DIM; ++c) {
      H[r * DIM + c] = sums[s];
      H[c * DIM + r] = sums[s];
      ++s;
    }
  for (int r = 0; r < DIM; ++r) g[r] = sums[NH + r];
  for (int k = 0; k < 49; ++k) res->H[k] = 0.0;
  for (int r = 0; r < DIM; ++r) {
    for (int c = 0; c < DIM; ++c) res->H[r * DIM + c] = H[r * DIM + c];
    res->g[r] = g[r];
  }
  res->err = sums[NS - 2];
  res->count = sums[NS - 1];
  int status = 0;
  if (sums[NS - 1] < (double)min_inliers * DIM) status = 1;
  // Cholesky H = L L^T
  for (int j = 0; j < DIM && status == 0; ++j) {
    double d = H[j * DIM + j];
    for (int k = 0; k < j; ++k) d -= L[j * DIM + k] * L[j * DIM + k];
    if (!(d > 0.0)) {
      status = 2;
      break;
    }
    const double ljj = sqrt(d);
    L[j * DIM + j] = ljj;
    for (int i = j + 1; i < DIM; ++i) {
      double v = H[i * DIM + j];
      for (int k = 0; k < j; ++k) v -= L[i * DIM + k] * L[j * DIM + k];
      L[i * DIM + j] = v / ljj;
    }
  }
  double step = 0.0;
  if (status == 0) {
    for (int i = 0; i < DIM; ++i) {   // L y = -g
      double v = -g[i];
      for (int k = 0; k < i; ++k) v -= L[i * DIM + k] * y[k];
      y[i] = v / L[i * DIM + i];
    }
    for (int i = DIM - 1; i >= 0; --i) {   // L^T xi = y
      double v = y[i];
      for (int k = i + 1; k < DIM; ++k) v -= L[k * DIM + i] * xi[k];
      xi[i] = v / L[i * DIM + i];
    }
    for (int i = 0; i < DIM; ++i) step += xi[i] * xi[i];
    step = sqrt(step);
    double E[16], T[16];
    exp_sim3(xi, DIM, E);
    for (int k = 0; k < 16; ++k) T[k] = pose[k];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        double v = 0.0;
        for (int k = 0; k < 4; ++k) v += E[4 * r + k] * T[4 * k + c];
        pose[4 * r + c] = v;
      }
  }
  for (int i = 0; i < 7; ++i) res->xi[i] = xi[i];
  res->step = step;
  res->status = status;
}

struct Scratch {
  double* pose = nullptr;
  float* partials = nullptr;
  ResultDev* res = nullptr;
  ResultDev* host_res = nullptr;
  double* host_pose = nullptr;
};

std::mutex g_mu;
std::vector<Scratch> g_scratch;

dtsdf_status get_scratch(Scratch** out) {
  int dev = 0;
  DTSDF_HIP(hipGetDevice(&dev));
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
  Scratch& s = g_scratch[dev];
  if (!s.pose) {
    if (hipMalloc(&s.pose, sizeof(double) * 16) != hipSuccess ||
        hipMalloc(&s.partials, sizeof(float) * kReduceBlocks * Sizes<7>::NS) != hipSuccess ||
        hipMalloc(&s.res, sizeof(ResultDev)) != hipSuccess ||
        hipHostMalloc(&s.host_res, sizeof(ResultDev), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&s.host_pose, sizeof(double) * 16, hipHostMallocDefault) != hipSuccess)
      return DTSDF_E_NOMEM;
  }
  *out = &s;
  return DTSDF_OK;
}

}  // namespace

extern "C" dtsdf_status icp_step(const dtsdf_image* live, const dtsdf_image* model, int32_t dim,
                                 const dtsdf_icp_params* p, double T[16], dtsdf_icp_result* out,
                                 void* stream) {
  if (!live || !model || !p || !T || (dim != 6 && dim != 7)) return DTSDF_E_INVAL;
  if (!live->vertex || !live->normal || !model->vertex || !model->normal) return DTSDF_E_INVAL;
  if (live->intr.width <= 0 || live->intr.height <= 0 || model->intr.width <= 0 ||
      model->intr.height <= 0 || !(model->intr.fx > 0) || !(model->intr.fy > 0) ||
      !(p->max_dist > 0) || !(p->max_angle_deg > 0) || p->min_inliers_per_dim < 0)
    return DTSDF_E_INVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  Scratch* s = nullptr;
  dtsdf_status st = get_scratch(&s);
  if (st != DTSDF_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  for (int k = 0; k < 16; ++k) s->host_pose[k] = T[k];
  DTSDF_HIP(hipMemcpyAsync(s->pose, s->host_pose, sizeof(double) * 16, hipMemcpyHostToDevice, hs));
  IcpArgs a;
  a.lv = live->vertex;
  a.ln = live->normal;
  a.lW = live->intr.width;
  a.lH = live->intr.height;
  a.mv = model->vertex;
  a.mn = model->normal;
  a.mmask = model->mask;
  a.mW = model->intr.width;
  a.mH = model->intr.height;
  a.fx = model->intr.fx;
  a.fy = model->intr.fy;
  a.cx = model->intr.cx;
  a.cy = model->intr.cy;
  a.max_dist2 = p->max_dist * p->max_dist;
  a.cos_angle = (float)cos((double)p->max_angle_deg * 3.14159265358979323846 / 180.0);
  a.weight_kind = p->weight;
  a.z_min = p->z_min;
  a.pose = s->pose;
  if (dim == 6) {
    hipLaunchKernelGGL(reduce_k<6>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, hs, a, s->partials);
    hipLaunchKernelGGL(solve_k<6>, dim3(1), dim3(64), 0, hs, s->partials, kReduceBlocks,
                       p->min_inliers_per_dim, s->pose, s->res);
  } else {
    hipLaunchKernelGGL(reduce_k<7>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, hs, a, s->partials);
    hipLaunchKernelGGL(solve_k<7>, dim3(1), dim3(64), 0, hs, s->partials, kReduceBlocks,
                       p->min_inliers_per_dim, s->pose, s->res);
  }
  DTSDF_HIP(hipGetLastError());
  DTSDF_HIP(hipMemcpyAsync(s->host_res, s->res, sizeof(ResultDev), hipMemcpyDeviceToHost, hs));
  DTSDF_HIP(hipMemcpyAsync(s->host_pose, s->pose, sizeof(double) * 16, hipMemcpyDeviceToHost, hs));
  DTSDF_HIP(hipStreamSynchronize(hs));
  const ResultDev& r = *s->host_res;
  if (out) {
    for (int i = 0; i < 7; ++i) out->xi[i] = r.xi[i];
    for (int i = 0; i < 49; ++i) out->H[i] = r.H[i];
    for (int i = 0; i < 7; ++i) out->g[i] = r.g[i];
    out->error = r.err;
    out->inliers = (int64_t)r.count;
    out->step_norm = r.step;
  }
  if (r.status != 0) return DTSDF_E_DEGENERATE;
  for (int k = 0; k < 16; ++k) T[k] = s->host_pose[k];
  return DTSDF_OK;
}
