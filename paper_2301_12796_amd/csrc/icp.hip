// Point-to-plane ICP step in SE(3) and Sim(3) (Sec. 5 and Sec. 6).
//
//   reduce_k<DIM>  per live pixel: transform, projective association, rejection, residual
//                  r = <q - y, n> and Jacobian J = (-n, -(y x n)[, -<n, y>]), plus, for
//                  combined ICP, the photometric residual against a reference grey image
//                  warped through T_RS, weighted by lambda (Sec. 5.2, 5.3); every thread
//                  sums a fixed strided subset of pixels in float32 (optionally with Neumaier
//                  compensation, merged by TwoSum), the workgroup folds its four waves with
//                  xor shuffles and a fixed-order LDS pass, and writes one partial vector.
//                  No atomics: the result is bitwise reproducible (the paper replaced atomic
//                  block sums for exactly this reason, Sec. 5).
//   Requests are reduced in 128 fixed pixel chunks (one workgroup each), so the summation
//   order of a request does not depend on what else is in its batch: a request's result is
//   bitwise the same alone (icp_step) and batched (icp_step_batch).
//   solve_k<DIM>   one workgroup: float64 sum of the partials in chunk order, Cholesky
//                  factorisation of H (eq. ICP_Hessian; the factor 2 cancels), xi = -H^-1 g
//                  (eq. ICP_solution), exp(xi) in closed form and T <- exp(xi) T
//                  (eq. deltaT_update), all on the device.
#include <cstring>
#include <algorithm>
#include <mutex>
#include <vector>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

constexpr int kChunks = 128;          // fixed pixel chunks per request (reduction order)
static_assert(kChunks % 16 == 0, "the solve sums chunks sixteen at a time");
constexpr int kReduceThreads = 512;

template <int DIM>
struct Sizes {
  static constexpr int NH = DIM * (DIM + 1) / 2;
  // H upper triangle, g, error, geometric count, photometric count
  static constexpr int NS = NH + DIM + 3;
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
  // photometric term (photo != 0): live grey values (live size), reference grey image,
  // its intrinsics, the model -> reference transform (rows of R | t) and the term's weight
  // and outlier threshold
  int photo;
  const float* li;
  const float* ri;
  int rW, rH;
  float rfx, rfy, rcx, rcy;
  float trs[12];
  float lambda, max_ierr;
};

constexpr int kNSMax = 7 * 8 / 2 + 7 + 3;   // partial sums of a 7-dof request

// Device descriptor of one registration request of a batch.
struct IcpJob {
  IcpArgs a;
  int dim;
  int compensated;
  int min_inliers;
  int pad;
  double min_step;
  int32_t* active;               // step only while *active != 0 (may be null: always)
  dtsdf_icp_result* result;      // may be null
};

// Error-free sum of two floats (Knuth's TwoSum): a + b = s + e exactly.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Running sum with Neumaier's compensation term.
struct CSum {
  float s, c;
  __device__ void add(float x) {
    const float t = s + x;
    c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ void merge(float s2, float c2) {
    float t, e;
    two_sum(s, s2, t, e);
    c = c + c2 + e;
    s = t;
  }
};

// Plain float32 accumulator with the same interface (compensation always zero).
struct PSum {
  float s, c;
  __device__ void add(float x) { s += x; }
  __device__ void merge(float s2, float) { s += s2; }
};

// Point-to-plane term of a live point y (model frame) with live normal nl: projective
// association, rejection, r = <q - y, n> and J = (-n, -(y x n)[, -<n, y>]) (eq. geometric_ICP,
// eq. ICP_geometric_dx; Sim(3): eq. sim3_derivative).  False if rejected.
template <int DIM>
__device__ inline bool geometric_term(const IcpArgs& a, bool has_normal, float nlx, float nly,
                                      float nlz, const float* R, const float* y, size_t MHW,
                                      float* J, float& res) {
  if (!has_normal || !(y[2] > 0.f)) return false;
  float nr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) nr[k] = R[3 * k] * nlx + R[3 * k + 1] * nly + R[3 * k + 2] * nlz;
  const float inr = 1.f / sqrtf(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
  const float uf = a.fx * y[0] / y[2] + a.cx;
  const float vf = a.fy * y[1] / y[2] + a.cy;
  const float ur = floorf(uf + 0.5f), vr = floorf(vf + 0.5f);
  if (!(ur >= 0.f && vr >= 0.f && ur < (float)a.mW && vr < (float)a.mH)) return false;
  const size_t mi = (size_t)vr * a.mW + (size_t)ur;
  if (a.mmask && !a.mmask[mi]) return false;
  const float n[3] = {a.mn[mi], a.mn[MHW + mi], a.mn[2 * MHW + mi]};
  if (!a.mmask && n[0] == 0.f && n[1] == 0.f && n[2] == 0.f) return false;
  const float d[3] = {a.mv[mi] - y[0], a.mv[MHW + mi] - y[1], a.mv[2 * MHW + mi] - y[2]};
  if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > a.max_dist2) return false;
  if ((n[0] * nr[0] + n[1] * nr[1] + n[2] * nr[2]) * inr < a.cos_angle) return false;
  res = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
  J[0] = -n[0];
  J[1] = -n[1];
  J[2] = -n[2];
  J[3] = -(y[1] * n[2] - y[2] * n[1]);
  J[4] = -(y[2] * n[0] - y[0] * n[2]);
  J[5] = -(y[0] * n[1] - y[1] * n[0]);
  if (DIM == 7) J[DIM - 1] = -(n[0] * y[0] + n[1] * y[1] + n[2] * y[2]);
  return true;
}

// Central difference of the reference image along x at pixel (u, v), zero on the border
// columns; the same along y.
__device__ inline float grad_u(const IcpArgs& a, int u, int v) {
  if (u <= 0 || u >= a.rW - 1) return 0.f;
  const float* row = a.ri + (size_t)v * a.rW;
  return 0.5f * (row[u + 1] - row[u - 1]);
}
__device__ inline float grad_v(const IcpArgs& a, int u, int v) {
  if (v <= 0 || v >= a.rH - 1) return 0.f;
  return 0.5f * (a.ri[(size_t)(v + 1) * a.rW + u] - a.ri[(size_t)(v - 1) * a.rW + u]);
}

// Photometric term of live pixel i with model-frame point y (eq. keyframe_icp): the point is
// taken to the reference camera by T_RS, projected to (u, v) in [1, W - 2] x [1, H - 2], the
// reference grey value and its central-difference gradient are interpolated bilinearly and
// r = I_live(i) - I_ref(u, v) with |r| <= max_ierr.  J is the derivative of r:
// -grad I . d(u, v)/da . R(T_RS) [I | -y^] (eq. keyframe_icp_derivative, eq. wedge_operator,
// eq. projection_dx with -x/z^2), Sim(3) scale column -grad I . d(u, v)/da . R(T_RS) y.
template <int DIM>
__device__ inline bool photometric_term(const IcpArgs& a, size_t i, const float* y, float* J,
                                        float& res) {
  const float* T = a.trs;
  const float ax = T[0] * y[0] + T[1] * y[1] + T[2] * y[2] + T[3];
  const float ay = T[4] * y[0] + T[5] * y[1] + T[6] * y[2] + T[7];
  const float az = T[8] * y[0] + T[9] * y[1] + T[10] * y[2] + T[11];
  if (!(az > 0.f)) return false;
  const float iz = 1.f / az;
  const float u = a.rfx * ax * iz + a.rcx, v = a.rfy * ay * iz + a.rcy;
  if (!(u >= 1.f && u <= (float)(a.rW - 2) && v >= 1.f && v <= (float)(a.rH - 2))) return false;
  const int u0 = (int)floorf(u), v0 = (int)floorf(v);
  const float fu = u - (float)u0, fv = v - (float)v0;
  const float w00 = (1.f - fu) * (1.f - fv), w10 = fu * (1.f - fv), w01 = (1.f - fu) * fv,
              w11 = fu * fv;
  const float* r0 = a.ri + (size_t)v0 * a.rW;
  const float* r1 = r0 + a.rW;
  const float Ik = w00 * r0[u0] + w10 * r0[u0 + 1] + w01 * r1[u0] + w11 * r1[u0 + 1];
  res = a.li[i] - Ik;
  if (!(fabsf(res) <= a.max_ierr)) return false;
  const float gx = w00 * grad_u(a, u0, v0) + w10 * grad_u(a, u0 + 1, v0) +
                   w01 * grad_u(a, u0, v0 + 1) + w11 * grad_u(a, u0 + 1, v0 + 1);
  const float gy = w00 * grad_v(a, u0, v0) + w10 * grad_v(a, u0 + 1, v0) +
                   w01 * grad_v(a, u0, v0 + 1) + w11 * grad_v(a, u0 + 1, v0 + 1);
  // dI/da = gx d u/da + gy d v/da, then c = dI/da R(T_RS) (derivative with respect to y)
  const float da0 = gx * a.rfx * iz, da1 = gy * a.rfy * iz;
  const float da2 = -(gx * a.rfx * ax + gy * a.rfy * ay) * iz * iz;
  const float c0 = da0 * T[0] + da1 * T[4] + da2 * T[8];
  const float c1 = da0 * T[1] + da1 * T[5] + da2 * T[9];
  const float c2 = da0 * T[2] + da1 * T[6] + da2 * T[10];
  J[0] = -c0;
  J[1] = -c1;
  J[2] = -c2;
  J[3] = -(y[1] * c2 - y[2] * c1);
  J[4] = -(y[2] * c0 - y[0] * c2);
  J[5] = -(y[0] * c1 - y[1] * c0);
  if (DIM == 7) J[DIM - 1] = -(c0 * y[0] + c1 * y[1] + c2 * y[2]);
  return true;
}

// Reduces the pixels of one chunk of a request into out[NS][2] (sum, compensation); called by
// all threads of a 256-thread workgroup.
template <int DIM, class Acc>
__device__ void reduce_chunk(const IcpArgs& a, int chunk, float* __restrict__ out) {
  constexpr int NS = Sizes<DIM>::NS;
  constexpr int NH = Sizes<DIM>::NH;
  Acc acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = Acc{0.f, 0.f};
  float R[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R[3 * r + c] = (float)a.pose[4 * r + c];
    t[r] = (float)a.pose[4 * r + 3];
  }
  const size_t LHW = (size_t)a.lW * a.lH;
  const size_t MHW = (size_t)a.mW * a.mH;
  const size_t per = (LHW + kChunks - 1) / kChunks;
  const size_t begin = (size_t)chunk * per, end = begin + per < LHW ? begin + per : LHW;
  for (size_t i = begin + threadIdx.x; i < end; i += kReduceThreads) {
    const float px = a.lv[i], py = a.lv[LHW + i], pz = a.lv[2 * LHW + i];
    const float nlx = a.ln[i], nly = a.ln[LHW + i], nlz = a.ln[2 * LHW + i];
    const bool has_normal = !(nlx == 0.f && nly == 0.f && nlz == 0.f);
    if (!has_normal && !(a.photo && pz > 0.f)) continue;
    float y[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] = R[3 * k] * px + R[3 * k + 1] * py + R[3 * k + 2] * pz + t[k];
    float w = 1.f;
    if (a.weight_kind == DTSDF_ICP_W_DEPTH) {
      const float zz = pz + (1.f - a.z_min);       // eq. ICP_weight
      w = 1.f / (zz * zz);
    }
    float J[DIM], res = 0.f;
    if (geometric_term<DIM>(a, has_normal, nlx, nly, nlz, R, y, MHW, J, res)) {
      int s = 0;
#pragma unroll
      for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = r; c < DIM; ++c) acc[s++].add(w * J[r] * J[c]);
#pragma unroll
      for (int r = 0; r < DIM; ++r) acc[NH + r].add(w * J[r] * res);
      acc[NH + DIM].add(w * res * res);
      acc[NH + DIM + 1].add(1.f);
    }
    if (a.photo && pz > 0.f && photometric_term<DIM>(a, i, y, J, res)) {
      const float lw = a.lambda * w;   // eq. combined_icp: E_geom + lambda E_photo
      int s = 0;
#pragma unroll
      for (int r = 0; r < DIM; ++r)
#pragma unroll
        for (int c = r; c < DIM; ++c) acc[s++].add(lw * J[r] * J[c]);
#pragma unroll
      for (int r = 0; r < DIM; ++r) acc[NH + r].add(lw * J[r] * res);
      acc[NH + DIM].add(lw * res * res);
      acc[NH + DIM + 2].add(1.f);
    }
  }
  // fixed-order tree: xor shuffles within the wave, then the waves in LDS order
  __shared__ float lds[kReduceThreads / 64][NS][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    Acc v = acc[s];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const float s2 = __shfl_xor(v.s, off, 64), c2 = __shfl_xor(v.c, off, 64);
      v.merge(s2, c2);
    }
    if (lane == 0) {
      lds[wave][s][0] = v.s;
      lds[wave][s][1] = v.c;
    }
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    Acc v{lds[0][threadIdx.x][0], lds[0][threadIdx.x][1]};
    for (int wv = 1; wv < kReduceThreads / 64; ++wv) v.merge(lds[wv][threadIdx.x][0], lds[wv][threadIdx.x][1]);
    out[threadIdx.x * 2] = v.s;
    out[threadIdx.x * 2 + 1] = v.c;
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

// Sum of partial sum `k` over the chunks, in chunk order (the fixed reduction order); the
// loads of 16 chunks are issued before their additions, which keep that order.
__device__ inline double sum_chunks(const float* __restrict__ partials, int k) {
  double v = 0.0;
  for (int c0 = 0; c0 < kChunks; c0 += 16) {
    float a[16], b[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      a[q] = partials[((size_t)(c0 + q) * kNSMax + k) * 2];
      b[q] = partials[((size_t)(c0 + q) * kNSMax + k) * 2 + 1];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) v += (double)a[q] + (double)b[q];
  }
  return v;
}

// Solves (A) xi = -g by Cholesky (A symmetric DIM x DIM); false if A is not positive definite.
template <int DIM>
__device__ bool cholesky_solve(const double* A, const double* g, double* xi) {
  double L[DIM * DIM], y[DIM];
  for (int jj = 0; jj < DIM; ++jj) {
    double d = A[jj * DIM + jj];
    for (int k = 0; k < jj; ++k) d -= L[jj * DIM + k] * L[jj * DIM + k];
    if (!(d > 0.0)) return false;
    const double ljj = sqrt(d);
    L[jj * DIM + jj] = ljj;
    for (int i = jj + 1; i < DIM; ++i) {
      double v = A[i * DIM + jj];
      for (int k = 0; k < jj; ++k) v -= L[i * DIM + k] * L[jj * DIM + k];
      L[i * DIM + jj] = v / ljj;
    }
  }
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
  return true;
}

// One Levenberg-Marquardt iteration with Madsen's damping (Sec. 7) for a request whose sums
// were taken at the candidate pose *j.a.pose: accept or reject the candidate by the gain
// ratio, then step from the accepted pose, (H + mu I) h = -g, and write the next candidate.
template <int DIM>
__device__ void solve_lm_one(const float* __restrict__ partials, const IcpJob& j,
                             dtsdf_lm_state* st) {
  constexpr int NS = Sizes<DIM>::NS;
  constexpr int NH = Sizes<DIM>::NH;
  __shared__ double sums[kNSMax];
  if (threadIdx.x < NS) sums[threadIdx.x] = sum_chunks(partials, threadIdx.x);
  __syncthreads();
  if (threadIdx.x != 0) return;
  double H[DIM * DIM], g[DIM], h[7] = {0, 0, 0, 0, 0, 0, 0};
  int s = 0;
  for (int r = 0; r < DIM; ++r)
    for (int c = r; c < DIM; ++c) {
      H[r * DIM + c] = sums[s];
      H[c * DIM + r] = sums[s];
      ++s;
    }
  for (int r = 0; r < DIM; ++r) g[r] = sums[NH + r];
  const double F = sums[NH + DIM];
  const double* cand = j.a.pose;
  int status = sums[NH + DIM + 1] < (double)j.min_inliers * DIM ? 1 : 0;
  double step = 0.0;
  st->accepted = 0;
  if (status == 0) {
    bool acc = false;
    if (!st->started) {
      double dmax = 0.0;
      for (int r = 0; r < DIM; ++r) dmax = fmax(dmax, H[r * DIM + r]);
      st->started = 1;
      st->mu = st->tau * dmax;
      st->nu = 2.0;
      acc = true;
    } else {
      double pred = 0.0;   // h^T (mu h - g_acc): the predicted reduction of sum w r^2
      for (int r = 0; r < DIM; ++r) pred += st->h[r] * (st->mu * st->h[r] - st->g[r]);
      const double rho = pred > 0.0 ? (st->F - F) / pred : -1.0;
      if (rho > 0.0) {
        const double q = 2.0 * rho - 1.0;
        st->mu *= fmax(1.0 / 3.0, 1.0 - q * q * q);
        st->nu = 2.0;
        acc = true;
      } else {
        st->mu *= st->nu;
        st->nu *= 2.0;
      }
    }
    if (acc) {
      for (int k = 0; k < 49; ++k) st->H[k] = k < DIM * DIM ? H[k] : 0.0;
      for (int k = 0; k < 7; ++k) st->g[k] = k < DIM ? g[k] : 0.0;
      st->F = F;
      for (int k = 0; k < 16; ++k) st->T_acc[k] = cand[k];
      st->accepted = 1;
    }
    double A[DIM * DIM], ga[DIM];
    for (int k = 0; k < DIM * DIM; ++k) A[k] = st->H[k];
    for (int r = 0; r < DIM; ++r) {
      A[r * DIM + r] += st->mu;
      ga[r] = st->g[r];
    }
    if (cholesky_solve<DIM>(A, ga, h)) {
      for (int r = 0; r < DIM; ++r) {
        st->h[r] = h[r];
        step += h[r] * h[r];
      }
      step = sqrt(step);
      double E[16];
      exp_sim3(h, DIM, E);
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          double v = 0.0;
          for (int k = 0; k < 4; ++k) v += E[4 * r + k] * st->T_acc[4 * k + c];
          st->T[4 * r + c] = v;
        }
    } else {
      status = 2;
    }
  }
  if (j.result) {
    dtsdf_icp_result* res = j.result;
    for (int k = 0; k < 49; ++k) res->H[k] = 0.0;
    for (int k = 0; k < 7; ++k) res->g[k] = 0.0;
    for (int r = 0; r < DIM; ++r) {
      for (int c = 0; c < DIM; ++c) res->H[r * DIM + c] = H[r * DIM + c];
      res->g[r] = g[r];
    }
    for (int i = 0; i < 7; ++i) res->xi[i] = h[i];
    res->error = F;
    res->inliers = (int64_t)sums[NH + DIM + 1];
    res->photometric = (int32_t)sums[NH + DIM + 2];
    res->step_norm = step;
    res->status = status == 0 ? DTSDF_OK : DTSDF_E_DEGENERATE;
  }
}

template <int DIM>
__device__ void solve_one(const float* __restrict__ partials, const IcpJob& j) {
  constexpr int NS = Sizes<DIM>::NS;
  constexpr int NH = Sizes<DIM>::NH;
  __shared__ double sums[kNSMax];
  if (threadIdx.x < NS) sums[threadIdx.x] = sum_chunks(partials, threadIdx.x);
  __syncthreads();
  if (threadIdx.x != 0) return;
  // the lone solving lane keeps the factorisation in LDS (as private arrays indexed in
  // loops they would live in scratch memory)
  __shared__ double H[DIM * DIM], L[DIM * DIM];
  double g[DIM], y[DIM], xi[7] = {0, 0, 0, 0, 0, 0, 0};
  int s = 0;
  for (int r = 0; r < DIM; ++r)
    for (int c = r; c < DIM; ++c) {
      H[r * DIM + c] = sums[s];
      H[c * DIM + r] = sums[s];
      ++s;
    }
  for (int r = 0; r < DIM; ++r) g[r] = sums[NH + r];
  int status = 0;
  if (sums[NH + DIM + 1] < (double)j.min_inliers * DIM) status = 1;
  // Cholesky H = L L^T
  for (int jj = 0; jj < DIM && status == 0; ++jj) {
    double d = H[jj * DIM + jj];
    for (int k = 0; k < jj; ++k) d -= L[jj * DIM + k] * L[jj * DIM + k];
    if (!(d > 0.0)) {
      status = 2;
      break;
    }
    const double ljj = sqrt(d);
    L[jj * DIM + jj] = ljj;
    for (int i = jj + 1; i < DIM; ++i) {
      double v = H[i * DIM + jj];
      for (int k = 0; k < jj; ++k) v -= L[i * DIM + k] * L[jj * DIM + k];
      L[i * DIM + jj] = v / ljj;
    }
  }
  double step = 0.0;
  double* pose = const_cast<double*>(j.a.pose);
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
  if (j.result) {
    dtsdf_icp_result* res = j.result;
    for (int k = 0; k < 49; ++k) res->H[k] = 0.0;
    for (int k = 0; k < 7; ++k) res->g[k] = 0.0;
    for (int r = 0; r < DIM; ++r) {
      for (int c = 0; c < DIM; ++c) res->H[r * DIM + c] = H[r * DIM + c];
      res->g[r] = g[r];
    }
    for (int i = 0; i < 7; ++i) res->xi[i] = xi[i];
    res->error = sums[NH + DIM];
    res->inliers = (int64_t)sums[NH + DIM + 1];
    res->photometric = (int32_t)sums[NH + DIM + 2];
    res->step_norm = step;
    res->status = status == 0 ? DTSDF_OK : DTSDF_E_DEGENERATE;
  }
  if (j.active && (status != 0 || step < j.min_step)) *j.active = 0;
}

__global__ __launch_bounds__(kReduceThreads) void reduce_batch_k(const IcpJob* __restrict__ jobs,
                                                                 float* partials) {
  const int r = blockIdx.y, c = blockIdx.x;
  const IcpJob& j = jobs[r];
  if (j.active && *j.active == 0) return;
  float* out = partials + ((size_t)r * kChunks + c) * kNSMax * 2;
  if (j.dim == 6) {
    if (j.compensated) reduce_chunk<6, CSum>(j.a, c, out);
    else reduce_chunk<6, PSum>(j.a, c, out);
  } else {
    if (j.compensated) reduce_chunk<7, CSum>(j.a, c, out);
    else reduce_chunk<7, PSum>(j.a, c, out);
  }
}

__global__ __launch_bounds__(64) void solve_lm_k(const IcpJob* __restrict__ jobs,
                                                 const float* __restrict__ partials,
                                                 dtsdf_lm_state* st) {
  if (jobs[0].dim == 6) solve_lm_one<6>(partials, jobs[0], st);
  else solve_lm_one<7>(partials, jobs[0], st);
}

__global__ __launch_bounds__(64) void solve_batch_k(const IcpJob* __restrict__ jobs,
                                                    const float* __restrict__ partials) {
  const IcpJob& j = jobs[blockIdx.x];
  if (j.active && *j.active == 0) return;
  const float* p = partials + (size_t)blockIdx.x * kChunks * kNSMax * 2;
  if (j.dim == 6) solve_one<6>(p, j);
  else solve_one<7>(p, j);
}

bool make_job(const dtsdf_image* live, const dtsdf_image* model, const dtsdf_photo* ph,
              int32_t dim, const dtsdf_icp_params* p, double* pose, int32_t* active,
              double min_step, dtsdf_icp_result* result, IcpJob& j) {
  if (!live || !model || !p || !pose || (dim != 6 && dim != 7)) return false;
  if (!live->vertex || !live->normal || !model->vertex || !model->normal) return false;
  if (live->intr.width <= 0 || live->intr.height <= 0 || model->intr.width <= 0 ||
      model->intr.height <= 0 || !(model->intr.fx > 0) || !(model->intr.fy > 0) ||
      !(p->max_dist > 0) || !(p->max_angle_deg > 0) || p->min_inliers_per_dim < 0)
    return false;
  IcpArgs& a = j.a;
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
  a.pose = pose;
  a.photo = ph ? 1 : 0;
  a.li = nullptr;
  a.ri = nullptr;
  a.rW = a.rH = 0;
  a.rfx = a.rfy = a.rcx = a.rcy = 0.f;
  for (int k = 0; k < 12; ++k) a.trs[k] = 0.f;
  a.lambda = a.max_ierr = 0.f;
  if (ph) {
    if (!ph->live_intensity || !ph->ref_intensity || ph->ref_intr.width < 3 ||
        ph->ref_intr.height < 3 || !(ph->ref_intr.fx > 0) || !(ph->ref_intr.fy > 0) ||
        !(ph->lambda >= 0.f) || !(ph->max_error > 0.f))
      return false;
    a.li = ph->live_intensity;
    a.ri = ph->ref_intensity;
    a.rW = ph->ref_intr.width;
    a.rH = ph->ref_intr.height;
    a.rfx = ph->ref_intr.fx;
    a.rfy = ph->ref_intr.fy;
    a.rcx = ph->ref_intr.cx;
    a.rcy = ph->ref_intr.cy;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 4; ++c) a.trs[4 * r + c] = (float)ph->T_ref_model[4 * r + c];
    a.lambda = ph->lambda;
    a.max_ierr = ph->max_error;
  }
  j.dim = dim;
  j.compensated = p->compensated;
  j.min_inliers = p->min_inliers_per_dim;
  j.pad = 0;
  j.min_step = min_step;
  j.active = active;
  j.result = result;
  return true;
}

// Per-device scratch of the single-request entry point (device pose, flag, result and the
// partial sums), guarded by a mutex: icp_step is synchronous, so calls do not overlap.
struct Scratch {
  uint8_t* dev = nullptr;        // job | pose | active | result
  float* partials = nullptr;
  uint8_t* host = nullptr;       // pinned mirror of `dev`
};

constexpr size_t kOffPose = (sizeof(IcpJob) + 63) & ~(size_t)63;
constexpr size_t kOffActive = kOffPose + 16 * sizeof(double);
constexpr size_t kOffResult = (kOffActive + sizeof(int32_t) + 63) & ~(size_t)63;
constexpr size_t kOffLm = (kOffResult + sizeof(dtsdf_icp_result) + 63) & ~(size_t)63;
constexpr size_t kScratchBytes = kOffLm + sizeof(dtsdf_lm_state);

std::mutex g_mu;
std::vector<Scratch> g_scratch;

dtsdf_status get_scratch(Scratch** out) {
  int dev = 0;
  DTSDF_HIP(hipGetDevice(&dev));
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
  Scratch& s = g_scratch[dev];
  if (!s.dev) {
    if (hipMalloc(&s.dev, kScratchBytes) != hipSuccess ||
        hipMalloc(&s.partials, sizeof(float) * 2 * kChunks * kNSMax) != hipSuccess ||
        hipHostMalloc(&s.host, kScratchBytes, hipHostMallocDefault) != hipSuccess)
      return DTSDF_E_NOMEM;
  }
  *out = &s;
  return DTSDF_OK;
}

__global__ __launch_bounds__(256) void intensity_k(const uint8_t* __restrict__ rgb, size_t n,
                                                   float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint8_t* c = rgb + 3 * i;
  out[i] = (0.299f * (float)c[0] + 0.587f * (float)c[1] + 0.114f * (float)c[2]) * (1.f / 255.f);
}

__global__ __launch_bounds__(256) void mean2x2_k(const float* __restrict__ in, int W, int H,
                                                 float* __restrict__ out) {
  const int Wo = W / 2, Ho = H / 2;
  const int u = blockIdx.x * 16 + (threadIdx.x & 15), v = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (u >= Wo || v >= Ho) return;
  const float* r0 = in + (size_t)(2 * v) * W + 2 * u;
  const float* r1 = r0 + W;
  out[(size_t)v * Wo + u] = 0.25f * ((r0[0] + r0[1]) + (r1[0] + r1[1]));
}

// ---- allocation-free batched step -----------------------------------------------------
// Requests of icp_step_batch_iters_noalloc: their descriptors and partial sums live in one
// fixed device array of the library (each GPU holds its own copy until the process ends);
// the descriptors reach it as kernel arguments, so no host or device memory is allocated and
// no host buffer has to outlive the call.
constexpr int kNoAllocMaxRequests = 16;
constexpr size_t kNoAllocJobBytes = (sizeof(IcpJob) * kNoAllocMaxRequests + 255) & ~(size_t)255;
constexpr size_t kNoAllocBytes =
    kNoAllocJobBytes + sizeof(float) * 2 * kChunks * kNSMax * kNoAllocMaxRequests;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kJobsPerPut = 8;
struct JobPack {
  IcpJob job[kJobsPerPut];
};
static_assert(sizeof(JobPack) <= 3072, "a pack of descriptors fits the kernel arguments");
static_assert(sizeof(IcpJob) % 4 == 0, "descriptors are copied as 32-bit words");

// Writes `count` descriptors of the pack (a kernel argument) to dst.
__global__ __launch_bounds__(256) void put_jobs_k(IcpJob* dst, JobPack pack, int count) {
  const int words = count * (int)(sizeof(IcpJob) / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&pack);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < words; i += blockDim.x) d[i] = src[i];
}

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64] = {};

// Device address of `scratch` on the current device, taken once per device (in host code
// the array's name is not a device address).
dtsdf_status noalloc_scratch(uint8_t** out) {
  int dev = 0;
  DTSDF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return DTSDF_E_INVAL;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DTSDF_E_HIP;
    g_noalloc_ptr[dev] = p;
  }
  *out = static_cast<uint8_t*>(g_noalloc_ptr[dev]);
  return DTSDF_OK;
}

// Batches whose descriptors exceed a staging slot: a pinned block of their own, released
// once the stream has run the batch (the call waits for it).
dtsdf_status icp_batch_large(int32_t n, const dtsdf_icp_req* reqs, int32_t iterations,
                             hipStream_t hs) {
  const size_t jb = (sizeof(IcpJob) * n + 255) & ~(size_t)255;
  const size_t pb = sizeof(float) * 2 * kChunks * kNSMax * (size_t)n;
  IcpJob* jobs = nullptr;
  uint8_t* dev = nullptr;
  if (hipHostMalloc((void**)&jobs, sizeof(IcpJob) * n, hipHostMallocDefault) != hipSuccess)
    return DTSDF_E_NOMEM;
  dtsdf_status rs = DTSDF_OK;
  for (int r = 0; r < n; ++r)
    make_job(&reqs[r].live, &reqs[r].model, reqs[r].photo, reqs[r].dim, &reqs[r].params,
             reqs[r].pose, reqs[r].active, reqs[r].min_step, reqs[r].result, jobs[r]);
  if (hipMallocAsync((void**)&dev, jb + pb, hs) != hipSuccess) {
    rs = DTSDF_E_NOMEM;
  } else {
    if (hipMemcpyAsync(dev, jobs, sizeof(IcpJob) * n, hipMemcpyHostToDevice, hs) != hipSuccess) {
      rs = DTSDF_E_HIP;
    } else {
      const IcpJob* dj = reinterpret_cast<const IcpJob*>(dev);
      float* part = reinterpret_cast<float*>(dev + jb);
      for (int it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(reduce_batch_k, dim3(kChunks, n), dim3(kReduceThreads), 0, hs, dj, part);
        hipLaunchKernelGGL(solve_batch_k, dim3(n), dim3(64), 0, hs, dj, part);
      }
      if (hipGetLastError() != hipSuccess) rs = DTSDF_E_HIP;
    }
    if (hipFreeAsync(dev, hs) != hipSuccess && rs == DTSDF_OK) rs = DTSDF_E_HIP;
  }
  if (hipStreamSynchronize(hs) != hipSuccess && rs == DTSDF_OK) rs = DTSDF_E_HIP;
  (void)hipHostFree(jobs);
  return rs;
}

}  // namespace

extern "C" dtsdf_status dtsdf_intensity(const uint8_t* rgb, int32_t width, int32_t height,
                                        float* out, void* stream) {
  if (!rgb || !out || width <= 0 || height <= 0) return DTSDF_E_INVAL;
  const size_t n = (size_t)width * height;
  hipLaunchKernelGGL(intensity_k, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, rgb, n, out);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

extern "C" dtsdf_status dtsdf_intensity_downsample(const float* in, int32_t width,
                                                   int32_t height, float* out, void* stream) {
  if (!in || !out || width < 2 || height < 2) return DTSDF_E_INVAL;
  dim3 grd((width / 2 + 15) / 16, (height / 2 + 15) / 16);
  hipLaunchKernelGGL(mean2x2_k, grd, dim3(256), 0, (hipStream_t)stream, in, width, height, out);
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

extern "C" dtsdf_status icp_step(const dtsdf_image* live, const dtsdf_image* model, int32_t dim,
                                 const dtsdf_icp_params* p, double T[16], dtsdf_icp_result* out,
                                 void* stream) {
  return icp_step_rgb(live, model, nullptr, dim, p, T, out, stream);
}

extern "C" dtsdf_status icp_step_rgb(const dtsdf_image* live, const dtsdf_image* model,
                                     const dtsdf_photo* photo, int32_t dim,
                                     const dtsdf_icp_params* p, double T[16],
                                     dtsdf_icp_result* out, void* stream) {
  if (!T) return DTSDF_E_INVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  Scratch* s = nullptr;
  dtsdf_status st = get_scratch(&s);
  if (st != DTSDF_OK) return st;
  IcpJob job;
  if (!make_job(live, model, photo, dim, p, reinterpret_cast<double*>(s->dev + kOffPose),
                reinterpret_cast<int32_t*>(s->dev + kOffActive), 0.0,
                reinterpret_cast<dtsdf_icp_result*>(s->dev + kOffResult), job))
    return DTSDF_E_INVAL;
  hipStream_t hs = (hipStream_t)stream;
  std::memcpy(s->host, &job, sizeof(job));
  std::memcpy(s->host + kOffPose, T, 16 * sizeof(double));
  const int32_t one = 1;
  std::memcpy(s->host + kOffActive, &one, sizeof(one));
  DTSDF_HIP(hipMemcpyAsync(s->dev, s->host, kOffResult, hipMemcpyHostToDevice, hs));
  hipLaunchKernelGGL(reduce_batch_k, dim3(kChunks, 1), dim3(kReduceThreads), 0, hs,
                     reinterpret_cast<const IcpJob*>(s->dev), s->partials);
  hipLaunchKernelGGL(solve_batch_k, dim3(1), dim3(64), 0, hs,
                     reinterpret_cast<const IcpJob*>(s->dev), s->partials);
  DTSDF_HIP(hipGetLastError());
  DTSDF_HIP(hipMemcpyAsync(s->host + kOffPose, s->dev + kOffPose, kScratchBytes - kOffPose,
                           hipMemcpyDeviceToHost, hs));
  DTSDF_HIP(hipStreamSynchronize(hs));
  dtsdf_icp_result r;
  std::memcpy(&r, s->host + kOffResult, sizeof(r));
  if (out) *out = r;
  if (r.status != DTSDF_OK) return DTSDF_E_DEGENERATE;
  std::memcpy(T, s->host + kOffPose, 16 * sizeof(double));
  return DTSDF_OK;
}

extern "C" dtsdf_status icp_step_lm(const dtsdf_image* live, const dtsdf_image* model,
                                    const dtsdf_photo* photo, int32_t dim,
                                    const dtsdf_icp_params* p, dtsdf_lm_state* state,
                                    dtsdf_icp_result* out, void* stream) {
  if (!state || !(state->tau >= 0.0)) return DTSDF_E_INVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  Scratch* s = nullptr;
  dtsdf_status st = get_scratch(&s);
  if (st != DTSDF_OK) return st;
  IcpJob job;
  if (!make_job(live, model, photo, dim, p, reinterpret_cast<double*>(s->dev + kOffPose),
                reinterpret_cast<int32_t*>(s->dev + kOffActive), 0.0,
                reinterpret_cast<dtsdf_icp_result*>(s->dev + kOffResult), job))
    return DTSDF_E_INVAL;
  hipStream_t hs = (hipStream_t)stream;
  std::memcpy(s->host, &job, sizeof(job));
  std::memcpy(s->host + kOffPose, state->T, 16 * sizeof(double));
  const int32_t one = 1;
  std::memcpy(s->host + kOffActive, &one, sizeof(one));
  std::memcpy(s->host + kOffLm, state, sizeof(*state));
  DTSDF_HIP(hipMemcpyAsync(s->dev, s->host, kScratchBytes, hipMemcpyHostToDevice, hs));
  hipLaunchKernelGGL(reduce_batch_k, dim3(kChunks, 1), dim3(kReduceThreads), 0, hs,
                     reinterpret_cast<const IcpJob*>(s->dev), s->partials);
  hipLaunchKernelGGL(solve_lm_k, dim3(1), dim3(64), 0, hs,
                     reinterpret_cast<const IcpJob*>(s->dev), s->partials,
                     reinterpret_cast<dtsdf_lm_state*>(s->dev + kOffLm));
  DTSDF_HIP(hipGetLastError());
  DTSDF_HIP(hipMemcpyAsync(s->host + kOffResult, s->dev + kOffResult, kScratchBytes - kOffResult,
                           hipMemcpyDeviceToHost, hs));
  DTSDF_HIP(hipStreamSynchronize(hs));
  dtsdf_icp_result r;
  std::memcpy(&r, s->host + kOffResult, sizeof(r));
  if (out) *out = r;
  if (r.status != DTSDF_OK) return DTSDF_E_DEGENERATE;
  std::memcpy(state, s->host + kOffLm, sizeof(*state));
  return DTSDF_OK;
}

extern "C" dtsdf_status icp_step_batch_iters(int32_t n, const dtsdf_icp_req* reqs,
                                             int32_t iterations, void* stream);

extern "C" dtsdf_status icp_step_batch(int32_t n, const dtsdf_icp_req* reqs, void* stream) {
  return icp_step_batch_iters(n, reqs, 1, stream);
}

extern "C" dtsdf_status icp_step_batch_iters(int32_t n, const dtsdf_icp_req* reqs,
                                             int32_t iterations, void* stream) {
  if (n < 0 || (n > 0 && !reqs) || n > 65535 || iterations < 1 || iterations > 1000)
    return DTSDF_E_INVAL;
  if (n == 0) return DTSDF_OK;
  IcpJob probe;
  for (int r = 0; r < n; ++r)
    if (!make_job(&reqs[r].live, &reqs[r].model, reqs[r].photo, reqs[r].dim, &reqs[r].params,
                  reqs[r].pose, reqs[r].active, reqs[r].min_step, reqs[r].result, probe))
      return DTSDF_E_INVAL;
  hipStream_t hs = (hipStream_t)stream;
  const size_t jb = (sizeof(IcpJob) * n + 255) & ~(size_t)255;
  const size_t pb = sizeof(float) * 2 * kChunks * kNSMax * (size_t)n;
  // descriptors through a staging slot (pinned host memory that outlives the copy); the
  // partial sums in the slot's device block when they fit, else stream-ordered memory
  Stage* sg = nullptr;
  if (jb > kStageHostBytes) return icp_batch_large(n, reqs, iterations, hs);
  dtsdf_status rs = stage_acquire(&sg);
  if (rs != DTSDF_OK) return rs;
  IcpJob* jobs = reinterpret_cast<IcpJob*>(sg->host);
  for (int r = 0; r < n; ++r)
    make_job(&reqs[r].live, &reqs[r].model, reqs[r].photo, reqs[r].dim, &reqs[r].params,
             reqs[r].pose, reqs[r].active, reqs[r].min_step, reqs[r].result, jobs[r]);
  float* part = nullptr;
  bool own_part = false;
  if (jb + pb <= kStageDevBytes) {
    part = reinterpret_cast<float*>(sg->dev + jb);
  } else if (hipMallocAsync((void**)&part, pb, hs) == hipSuccess) {
    own_part = true;
  } else {
    rs = DTSDF_E_NOMEM;
  }
  if (rs == DTSDF_OK) {
    if (hipMemcpyAsync(sg->dev, sg->host, sizeof(IcpJob) * n, hipMemcpyHostToDevice, hs) !=
        hipSuccess) {
      rs = DTSDF_E_HIP;
    } else {
      const IcpJob* dj = reinterpret_cast<const IcpJob*>(sg->dev);
      // the descriptors hold device pointers to each request's pose and flag, so the same
      // launches repeated continue from the poses the previous ones wrote
      for (int it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(reduce_batch_k, dim3(kChunks, n), dim3(kReduceThreads), 0, hs, dj, part);
        hipLaunchKernelGGL(solve_batch_k, dim3(n), dim3(64), 0, hs, dj, part);
      }
      if (hipGetLastError() != hipSuccess) rs = DTSDF_E_HIP;
    }
  }
  if (own_part && hipFreeAsync(part, hs) != hipSuccess && rs == DTSDF_OK) rs = DTSDF_E_HIP;
  const dtsdf_status rr = stage_release(sg, hs);
  return rs != DTSDF_OK ? rs : rr;
}

namespace {
__global__ void set_flag_k(int32_t* flag) {
  if (threadIdx.x == 0) *flag = 1;
}
}  // namespace

extern "C" dtsdf_status dtsdf_level_intrinsics(const dtsdf_intrinsics* in, int32_t level,
                                               dtsdf_intrinsics* out) {
  if (!in || !out || level < 0 || level > 15 || in->width <= 0 || in->height <= 0)
    return DTSDF_E_INVAL;
  const double s = (double)(1 << level);
  dtsdf_intrinsics o;
  o.width = in->width >> level;
  o.height = in->height >> level;
  if (o.width <= 0 || o.height <= 0) return DTSDF_E_INVAL;
  o.fx = (float)((double)in->fx / s);
  o.fy = (float)((double)in->fy / s);
  o.cx = (float)(((double)in->cx + 0.5) / s - 0.5);
  o.cy = (float)(((double)in->cy + 0.5) / s - 0.5);
  *out = o;
  return DTSDF_OK;
}

extern "C" dtsdf_status dtsdf_icp_pyramid(int32_t levels, const dtsdf_icp_req* reqs,
                                          const int32_t* iterations, void* stream) {
  if (levels < 1 || levels > 16 || !reqs || !iterations) return DTSDF_E_INVAL;
  for (int l = 0; l < levels; ++l)
    if (reqs[l].pose != reqs[0].pose || !reqs[l].active || iterations[l] < 0 ||
        iterations[l] > 1000)
      return DTSDF_E_INVAL;
  hipStream_t hs = (hipStream_t)stream;
  for (int l = levels - 1; l >= 0; --l) {
    if (iterations[l] == 0) continue;
    // every level starts afresh: its convergence flag is raised on the device, in stream
    // order after the previous level's steps
    hipLaunchKernelGGL(set_flag_k, dim3(1), dim3(64), 0, hs, reqs[l].active);
    DTSDF_HIP(hipGetLastError());
    const dtsdf_status st = icp_step_batch_iters(1, &reqs[l], iterations[l], stream);
    if (st != DTSDF_OK) return st;
  }
  return DTSDF_OK;
}

extern "C" dtsdf_status icp_step_batch_iters_noalloc(int32_t n, const dtsdf_icp_req* reqs,
                                                     int32_t iterations, void* stream) {
  if (n < 0 || (n > 0 && !reqs) || n > kNoAllocMaxRequests || iterations < 1 ||
      iterations > 1000)
    return DTSDF_E_INVAL;
  if (n == 0) return DTSDF_OK;
  JobPack packs[(kNoAllocMaxRequests + kJobsPerPut - 1) / kJobsPerPut];
  for (int r = 0; r < n; ++r)
    if (!make_job(&reqs[r].live, &reqs[r].model, reqs[r].photo, reqs[r].dim, &reqs[r].params,
                  reqs[r].pose, reqs[r].active, reqs[r].min_step, reqs[r].result,
                  packs[r / kJobsPerPut].job[r % kJobsPerPut]))
      return DTSDF_E_INVAL;
  uint8_t* base = nullptr;
  const dtsdf_status s0 = noalloc_scratch(&base);
  if (s0 != DTSDF_OK) return s0;
  hipStream_t hs = (hipStream_t)stream;
  IcpJob* dj = reinterpret_cast<IcpJob*>(base);
  float* part = reinterpret_cast<float*>(base + kNoAllocJobBytes);
  for (int b = 0; b < n; b += kJobsPerPut)
    hipLaunchKernelGGL(put_jobs_k, dim3(1), dim3(256), 0, hs, dj + b, packs[b / kJobsPerPut],
                       std::min(kJobsPerPut, n - b));
  // every partial sum a solve reads is written by the reduce before it, so nothing of the
  // previous call's contents is used
  for (int it = 0; it < iterations; ++it) {
    hipLaunchKernelGGL(reduce_batch_k, dim3(kChunks, n), dim3(kReduceThreads), 0, hs, dj, part);
    hipLaunchKernelGGL(solve_batch_k, dim3(n), dim3(64), 0, hs, dj, part);
  }
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}
