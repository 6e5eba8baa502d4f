// Plain FP64 CPU oracle of Directional-TSDF integration and rendering.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
// benchmark load this library.  It shares no code, header, table or helper with the HIP
// library; both sides only consume the seeded inputs of the `synth` package.
//
// Every function follows the paper step by step in double precision, with no blocking,
// fusion or reordering beyond what the definitions state:
//   * voxel tuple (d, w_d, c, w_c) and six directional TSDFs        -- Sec. 3
//   * direction membership weight w_dir                                -- Sec. 3, eq. direction_weight
//   * fusion weight w_d = w_depth * w_angle * w_dir                    -- Sec. 3, eq. combined_fusion_weight
//   * colour weight w_c = w_d (1 - min(1, |p - x| / tau))              -- Sec. 3, eq. color_weight
//   * point-to-plane signed distance, normalised and clamped           -- Sec. 3, eq. point-to-plane
//   * free-space carving with the two-pixel depth-jump guard           -- Sec. 3
//   * voxel-projection fusion                                          -- Sec. 3
//   * blocks of 8^3 voxels keyed by (x, y, z, D)                       -- Sec. 7
//   * ray casting: regular probing, then a bracketed refinement        -- Sec. 4
//   * combination weight w_dir(n^D) <n^D, -r> w_d^D                    -- Sec. 4, eq. combine_weight
//   * gradient-free fallback w^D <v^D, -r>                             -- Sec. 4, eq. combine_tsdf_weight
// Readings where the paper is silent or garbled are listed in the design notes and repeated
// at the point of use below.
//
// Build: g++ -O2 -fopenmp -shared -fPIC dtsdf_oracle.cpp -o liboracle.so
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <omp.h>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace {

constexpr int kB = 8;                 // voxels per block edge (Sec. 7)
constexpr int kVox = kB * kB * kB;    // voxels per block
constexpr double kPi = 3.14159265358979323846;

// Direction order X+, X-, Y+, Y-, Z+, Z- with axis vectors v^D (Sec. 3).
const double kAxis[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

struct Params {
  double voxel;        // voxel edge s [m]
  double tau;          // truncation distance [m]
  double theta;        // angular threshold, in (pi/4, pi/2]
  double w_carve;      // constant free-space weight (value not given in the paper)
  double w_max;        // weight cap (not given)
  double w_min;        // updates with fusion weight below this are skipped
  double step;         // lattice step of the ray march (not given)
  int32_t dense;       // 1: fixed block range allocated up front, no growth
  int32_t dense_lo[3];
  int32_t dense_hi[3];
  int32_t with_color;
  int32_t single_direction;  // control: one direction with w_dir = 1 (a regular TSDF)
  int32_t sdf_fmt;           // 0 float, 1 float16 code, 2 int16 code scaled by the truncation
  int32_t w_fmt;             // 0 float, 1 uint8 code q, w = q^2 / 1024
};

struct Key {
  int32_t x, y, z, d;
  bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z && d == o.d; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = (uint64_t)(uint32_t)k.x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.y * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.z * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.d + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};
struct BKey {
  int32_t x, y, z;
  bool operator==(const BKey& o) const { return x == o.x && y == o.y && z == o.z; }
};
struct BKeyHash {
  size_t operator()(const BKey& k) const { return KeyHash()(Key{k.x, k.y, k.z, 0}); }
};

struct Brick {
  double sdf[kVox];
  double w[kVox];
  uint8_t rgb[kVox][3];
  double wc[kVox];
  uint8_t border[kVox];   // 1: some decision for this voxel sat on a threshold (see below)
};

struct Map {
  Params p;
  std::unordered_map<Key, int, KeyHash> index;   // (block, D) -> brick ordinal
  std::unordered_set<BKey, BKeyHash> blocks;     // blocks with at least one direction
  std::vector<Key> keys;
  std::deque<Brick> bricks;    // stable addresses, no reallocation copies
};

inline int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

int add_brick(Map& m, const Key& k) {
  auto it = m.index.find(k);
  if (it != m.index.end()) return it->second;
  int id = (int)m.bricks.size();
  m.bricks.emplace_back();
  Brick& b = m.bricks.back();
  std::memset(&b, 0, sizeof(Brick));
  m.index.emplace(k, id);
  m.keys.push_back(k);
  m.blocks.insert(BKey{k.x, k.y, k.z});
  return id;
}

// Direction membership weight (Sec. 3, eq. direction_weight).  The printed fraction does not
// meet the properties the paper states next to it (zero beyond theta, one in the exclusive
// zone, linear across the whole blend zone); the clamped-linear function with exactly those
// properties is used: the blend zone between two neighbouring axes is [pi/2 - theta, theta].
double w_dir(const Params& p, const double n[3], int d) {
  if (p.single_direction) return d == 0 ? 1.0 : 0.0;
  double c = n[0] * kAxis[d][0] + n[1] * kAxis[d][1] + n[2] * kAxis[d][2];
  c = std::min(1.0, std::max(-1.0, c));
  double a = std::acos(c);
  double v = (p.theta - a) / (2.0 * p.theta - 0.5 * kPi);
  return std::min(1.0, std::max(0.0, v));
}

// w_dir with `margin` added before clamping (classification of threshold cases only).
double w_dir_shifted(const Params& p, const double n[3], int d, double margin) {
  double c = n[0] * kAxis[d][0] + n[1] * kAxis[d][1] + n[2] * kAxis[d][2];
  c = std::min(1.0, std::max(-1.0, c));
  double v = (p.theta - std::acos(c)) / (2.0 * p.theta - 0.5 * kPi) + margin;
  return std::min(1.0, std::max(0.0, v));
}

// Margin of the w_dir > 0 decision: angle distance to theta (radians).
double w_dir_margin(const Params& p, const double n[3], int d) {
  double c = n[0] * kAxis[d][0] + n[1] * kAxis[d][1] + n[2] * kAxis[d][2];
  c = std::min(1.0, std::max(-1.0, c));
  return std::fabs(std::acos(c) - p.theta);
}

inline double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ---------------------------------------------------------------------------------------
// Integration (Sec. 3)
// ---------------------------------------------------------------------------------------

struct Frame {
  int W, H;
  std::vector<double> P;      // camera-frame points, 3 per pixel
  std::vector<double> N;      // camera-frame unit normals facing the camera
  std::vector<uint8_t> pv;    // depth valid
  std::vector<uint8_t> nv;    // normal valid
};

// Back-projection (Sec. 6, eq. reprojection) and cross-product normals (Sec. 7): the normal
// of pixel (u, v) is the normalised cross product of the central differences in x and y,
// oriented towards the camera; it is invalid unless the pixel and its four neighbours have
// depth.
Frame make_frame(const float* depth, int W, int H, double fx, double fy, double cx, double cy,
                 double depth_scale) {
  Frame f;
  f.W = W;
  f.H = H;
  f.P.assign((size_t)W * H * 3, 0.0);
  f.N.assign((size_t)W * H * 3, 0.0);
  f.pv.assign((size_t)W * H, 0);
  f.nv.assign((size_t)W * H, 0);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      size_t i = (size_t)v * W + u;
      double z = (double)depth[i] * depth_scale;
      if (!(z > 0.0) || !std::isfinite(z)) continue;
      f.P[3 * i + 0] = z * (u - cx) / fx;
      f.P[3 * i + 1] = z * (v - cy) / fy;
      f.P[3 * i + 2] = z;
      f.pv[i] = 1;
    }
  for (int v = 1; v + 1 < H; ++v)
    for (int u = 1; u + 1 < W; ++u) {
      size_t i = (size_t)v * W + u;
      size_t l = i - 1, r = i + 1, t = i - W, b = i + W;
      if (!(f.pv[i] && f.pv[l] && f.pv[r] && f.pv[t] && f.pv[b])) continue;
      double dx[3], dy[3], n[3];
      for (int k = 0; k < 3; ++k) {
        dx[k] = f.P[3 * r + k] - f.P[3 * l + k];
        dy[k] = f.P[3 * b + k] - f.P[3 * t + k];
      }
      n[0] = dx[1] * dy[2] - dx[2] * dy[1];
      n[1] = dx[2] * dy[0] - dx[0] * dy[2];
      n[2] = dx[0] * dy[1] - dx[1] * dy[0];
      double len = std::sqrt(dot3(n, n));
      if (!(len > 0.0)) continue;
      double s = (dot3(n, &f.P[3 * i]) > 0.0) ? -1.0 / len : 1.0 / len;
      for (int k = 0; k < 3; ++k) f.N[3 * i + k] = n[k] * s;
      f.nv[i] = 1;
    }
  return f;
}

// Replaces the frame's cross-product normals by the caller's (camera frame, three per
// pixel, all zero = none; Sec. 7 filters the normals before use); a normal counts only where
// the depth is valid.
void override_normals(Frame& f, const double* normals) {
  if (!normals) return;
  for (size_t i = 0; i < (size_t)f.W * f.H; ++i) {
    const double* n = normals + 3 * i;
    const bool ok = f.pv[i] && (n[0] != 0.0 || n[1] != 0.0 || n[2] != 0.0);
    for (int k = 0; k < 3; ++k) f.N[3 * i + k] = ok ? n[k] : 0.0;
    f.nv[i] = ok ? 1 : 0;
  }
}

void running_average(double& val, double& w, double x, double wx, double w_max) {
  val = (val * w + x * wx) / (w + wx);
  w = std::min(w + wx, w_max);
}

// Round half to even to a multiple of `quantum`; `tie` is set when x lies within `tol`
// quanta of a rounding boundary (a float32 implementation, whose running averages carry a
// few float32 ulps of error, may round the other way there).
double round_to(double x, double quantum, double tol, bool* tie) {
  const double y = x / quantum;
  if (std::fabs(y - std::floor(y) - 0.5) < tol) *tie = true;
  return std::nearbyint(y) * quantum;
}

// Stored form of a distance: float16 keeps 10 fraction bits in the binade of x (spacing
// 2^-24 below the smallest normal); int16 keeps the code q = round(32767 d), which decodes
// as q times the float32 scale 1/32767 (the product rounded to float32).
double store_sdf(const Params& p, double d, bool* tie) {
  if (p.sdf_fmt == 1) {
    const double ax = std::fabs(d);
    if (ax == 0.0) return d;
    int e;
    std::frexp(ax, &e);
    return round_to(d, std::ldexp(1.0, std::max(e - 11, -24)), 1e-3, tie);
  }
  if (p.sdf_fmt == 2) {
    const double q = std::min(32767.0, std::max(-32767.0, round_to(d * 32767.0, 1.0, 5e-2, tie)));
    return (double)((float)q * (1.0f / 32767.0f));
  }
  return d;
}

// Stored form of a weight in the uint8 format: the code q = round-half-even(sqrt(1024 w)),
// at most 255, standing for w = q^2 / 1024 (a square-law code: its step (2 q + 1) / 1024
// is fine at small weights, so that carving and small fusion weights accumulate).  `tie`
// is set when 1024 w lies within 1e-3 steps of a rounding boundary (q + 1/2)^2.
double store_w(const Params& p, double w, bool* tie) {
  if (p.w_fmt != 1) return w;
  const double x = 1024.0 * std::max(0.0, w);
  // nearbyint rounds half to even; the square root of an exact boundary (c + 1/2)^2 is
  // exact, so ties go to the even code
  double q = std::nearbyint(std::sqrt(x));
  for (double c : {q - 1.0, q}) {   // the boundaries below and above q
    if (c < 0) continue;
    const double mid = c * c + c + 0.25;
    if (std::fabs(x - mid) < 1e-3 * (2.0 * c + 1.0)) *tie = true;
  }
  q = std::min(255.0, q);
  return q * q / 1024.0;
}

}  // namespace

extern "C" {

struct OrcStats {
  int64_t requests;         // (block, D) requests emitted by valid pixels
  int64_t borderline_req;   // requests whose block or direction decision sat on a threshold
  int64_t new_bricks;       // bricks added by this call
  int64_t updated;          // voxel updates (surface band)
  int64_t carved;           // voxel updates (free space)
};

void* orc_create(const Params* p) {
  Map* m = new Map();
  m->p = *p;
  if (p->dense) {
    for (int bz = p->dense_lo[2]; bz <= p->dense_hi[2]; ++bz)
      for (int by = p->dense_lo[1]; by <= p->dense_hi[1]; ++by)
        for (int bx = p->dense_lo[0]; bx <= p->dense_hi[0]; ++bx)
          for (int d = 0; d < (p->single_direction ? 1 : 6); ++d) add_brick(*m, Key{bx, by, bz, d});
  }
  return m;
}

void orc_destroy(void* h) { delete static_cast<Map*>(h); }

int64_t orc_num_bricks(void* h) { return (int64_t) static_cast<Map*>(h)->bricks.size(); }

// Allocation requests of one frame (Sec. 7: blocks are allocated for every point with a valid
// normal).  For each valid pixel and each direction with w_dir > 0, the blocks containing the
// J+1 evenly spaced points p + t r, t in [-tau, tau], J = ceil(2 tau / s), are requested
// (r: unit ray through the pixel).  A request is "borderline" when a point lies within 1e-9
// block units of a block face or the direction's angle is within 1e-6 rad of theta; for the
// latter case the blocks a direction just below the threshold would have requested are also
// listed, with alloc = 0, so that a comparison can accept either outcome.
static void collect_requests(const Map& m, const Frame& f, const double T[16],
                             std::vector<Key>& req, std::vector<uint8_t>& border,
                             std::vector<uint8_t>& alloc) {
  const Params& p = m.p;
  int J = (int)std::ceil(2.0 * p.tau / p.voxel - 1e-9);
  double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double t[3] = {T[3], T[7], T[11]};
  for (int v = 0; v < f.H; ++v)
    for (int u = 0; u < f.W; ++u) {
      size_t i = (size_t)v * f.W + u;
      if (!f.nv[i]) continue;
      double pw[3], nw[3], rw[3];
      const double* pc = &f.P[3 * i];
      const double* nc = &f.N[3 * i];
      for (int k = 0; k < 3; ++k) {
        pw[k] = R[3 * k] * pc[0] + R[3 * k + 1] * pc[1] + R[3 * k + 2] * pc[2] + t[k];
        nw[k] = R[3 * k] * nc[0] + R[3 * k + 1] * nc[1] + R[3 * k + 2] * nc[2];
      }
      double len = std::sqrt(dot3(pc, pc));
      for (int k = 0; k < 3; ++k)
        rw[k] = (R[3 * k] * pc[0] + R[3 * k + 1] * pc[1] + R[3 * k + 2] * pc[2]) / len;
      for (int d = 0; d < 6; ++d) {
        bool edge = !p.single_direction && w_dir_margin(p, nw, d) < 1e-6;
        bool on = w_dir(p, nw, d) > 0.0;
        if (!on && !edge) continue;
        for (int j = 0; j <= J; ++j) {
          double s = -p.tau + 2.0 * p.tau * j / J, q[3];
          bool bl = edge;
          for (int k = 0; k < 3; ++k) {
            q[k] = (pw[k] + s * rw[k]) / p.voxel / kB;
            double fr = q[k] - std::floor(q[k]);
            if (fr < 1e-9 || fr > 1.0 - 1e-9) bl = true;
          }
          req.push_back(Key{(int32_t)std::floor(q[0]), (int32_t)std::floor(q[1]),
                            (int32_t)std::floor(q[2]), d});
          border.push_back(bl ? 1 : 0);
          alloc.push_back(on ? 1 : 0);
        }
      }
    }
}

// Returns the requested (block, D) keys of one frame without changing the map:
// out_keys[4*i..] = (bx, by, bz, D), out_border[i] = borderline flag, out_alloc[i] = 1 if the
// request allocates (0: listed only as the other outcome of a borderline decision).
// Duplicates are kept.
int64_t orc_requests(void* h, const float* depth, int W, int H, double fx, double fy, double cx,
                     double cy, const double T[16], double depth_scale, int32_t* out_keys,
                     uint8_t* out_border, uint8_t* out_alloc, int64_t cap,
                     const double* normals) {
  Map& m = *static_cast<Map*>(h);
  Frame f = make_frame(depth, W, H, fx, fy, cx, cy, depth_scale);
  override_normals(f, normals);
  std::vector<Key> req;
  std::vector<uint8_t> border, alloc;
  collect_requests(m, f, T, req, border, alloc);
  int64_t n = (int64_t)req.size();
  for (int64_t i = 0; i < n && i < cap; ++i) {
    out_keys[4 * i + 0] = req[i].x;
    out_keys[4 * i + 1] = req[i].y;
    out_keys[4 * i + 2] = req[i].z;
    out_keys[4 * i + 3] = req[i].d;
    out_border[i] = border[i];
    out_alloc[i] = alloc[i];
  }
  return n;
}

// Fuse one depth (+colour) frame with known camera-to-world pose T (row-major 4x4).
// depth: HxW float32 metres before depth_scale, 0 = invalid.  rgb: HxWx3 or NULL.
void orc_integrate(void* h, const float* depth, const uint8_t* rgb, int W, int H, double fx,
                   double fy, double cx, double cy, const double T[16], double depth_scale,
                   OrcStats* st, const double* normals) {
  Map& m = *static_cast<Map*>(h);
  const Params& p = m.p;
  OrcStats s{};
  Frame f = make_frame(depth, W, H, fx, fy, cx, cy, depth_scale);
  override_normals(f, normals);
  double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double t[3] = {T[3], T[7], T[11]};

  // 1. allocation of the requested (block, D) bricks (sparse maps only)
  if (!p.dense) {
    std::vector<Key> req;
    std::vector<uint8_t> border, alloc;
    collect_requests(m, f, T, req, border, alloc);
    for (size_t i = 0; i < req.size(); ++i) {
      if (!alloc[i]) continue;
      s.requests++;
      s.borderline_req += border[i];
      size_t before = m.bricks.size();
      add_brick(m, req[i]);
      if (m.bricks.size() > before) s.new_bricks++;
    }
  }

  // world-frame points and normals of the frame
  std::vector<double> Pw((size_t)W * H * 3), Nw((size_t)W * H * 3);
  for (size_t i = 0; i < (size_t)W * H; ++i)
    for (int k = 0; k < 3; ++k) {
      Pw[3 * i + k] = R[3 * k] * f.P[3 * i] + R[3 * k + 1] * f.P[3 * i + 1] +
                      R[3 * k + 2] * f.P[3 * i + 2] + t[k];
      Nw[3 * i + k] = R[3 * k] * f.N[3 * i] + R[3 * k + 1] * f.N[3 * i + 1] +
                      R[3 * k + 2] * f.N[3 * i + 2];
    }

  // 2. voxel-projection fusion of every allocated voxel (Sec. 3)
  int64_t n_upd = 0, n_carve = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_upd, n_carve)
  for (int64_t bi = 0; bi < (int64_t)m.bricks.size(); ++bi) {
    Brick& B = m.bricks[bi];
    const Key k = m.keys[bi];
    const int D = k.d;
    for (int l = 0; l < kVox; ++l) {
      int lx = l % kB, ly = (l / kB) % kB, lz = l / (kB * kB);
      double x[3] = {(double)(k.x * kB + lx) * p.voxel, (double)(k.y * kB + ly) * p.voxel,
                     (double)(k.z * kB + lz) * p.voxel};
      double xr[3] = {x[0] - t[0], x[1] - t[1], x[2] - t[2]};
      double xc[3];
      for (int a = 0; a < 3; ++a) xc[a] = R[a] * xr[0] + R[3 + a] * xr[1] + R[6 + a] * xr[2];
      if (!(xc[2] > 0.0)) continue;
      double uf = fx * xc[0] / xc[2] + cx, vf = fy * xc[1] / xc[2] + cy;
      double ur = std::floor(uf + 0.5), vr = std::floor(vf + 0.5);
      if (ur < 0 || vr < 0 || ur >= W || vr >= H) continue;
      // nearest-pixel association: a voxel projecting within 1e-6 px of a pixel border is
      // borderline (another implementation may pick the neighbouring pixel)
      double fu = uf + 0.5 - ur, fv = vf + 0.5 - vr;
      bool bl = fu < 1e-6 || fu > 1 - 1e-6 || fv < 1e-6 || fv > 1 - 1e-6;
      int u = (int)ur, v = (int)vr;
      size_t pi = (size_t)v * W + u;
      if (!f.nv[pi]) {
        if (bl) B.border[l] = 1;
        continue;
      }
      const double* pw = &Pw[3 * pi];
      const double* nw = &Nw[3 * pi];
      // point-to-plane distance (Sec. 3, eq. point-to-plane), sign chosen so that positive
      // values lie in front of the surface: the normal faces the camera, so the printed
      // <p - x, n> is negated to <x - p, n>.
      double dd = ((x[0] - pw[0]) * nw[0] + (x[1] - pw[1]) * nw[1] + (x[2] - pw[2]) * nw[2]) /
                  p.tau;
      if (std::fabs(dd - 1.0) < 1e-6 || std::fabs(dd + 1.0) < 1e-6) bl = true;
      if (dd > 1.0) {
        // free space: carve with value 1 and a constant weight, no direction weight, unless a
        // valid depth within a two-pixel radius differs by more than tau (Sec. 3)
        double z0 = (double)depth[pi] * depth_scale;
        bool ok = true;
        for (int dv = -2; dv <= 2; ++dv)
          for (int du = -2; du <= 2; ++du) {
            int uu = u + du, vv = v + dv;
            if (uu < 0 || vv < 0 || uu >= W || vv >= H) continue;
            double z1 = (double)depth[(size_t)vv * W + uu] * depth_scale;
            if (!(z1 > 0.0)) continue;
            double jump = std::fabs(z1 - z0);
            if (std::fabs(jump - p.tau) < 1e-6 * p.tau) bl = true;
            if (jump > p.tau) ok = false;
          }
        if (ok && p.w_carve > 0.0) {
          running_average(B.sdf[l], B.w[l], 1.0, p.w_carve, p.w_max);
          B.sdf[l] = store_sdf(p, B.sdf[l], &bl);
          B.w[l] = store_w(p, B.w[l], &bl);
          n_carve++;
        }
        if (bl) B.border[l] = 1;
        continue;
      }
      if (dd < -1.0) {  // behind the band: no update
        if (bl) B.border[l] = 1;
        continue;
      }
      double wd_dir = w_dir(p, nw, D);
      if (!p.single_direction && w_dir_margin(p, nw, D) < 1e-6) bl = true;
      if (!(wd_dir > 0.0)) {
        if (bl) B.border[l] = 1;
        continue;
      }
      // w_d = w_depth * w_angle * w_dir (Sec. 3, eq. combined_fusion_weight); the paper omits
      // the parameters: w_depth = 1 and w_angle = max(0, <n, -r>) with r the unit ray from the
      // camera through the pixel.
      double rl = std::sqrt((pw[0] - t[0]) * (pw[0] - t[0]) + (pw[1] - t[1]) * (pw[1] - t[1]) +
                            (pw[2] - t[2]) * (pw[2] - t[2]));
      double cosang = -((pw[0] - t[0]) * nw[0] + (pw[1] - t[1]) * nw[1] +
                        (pw[2] - t[2]) * nw[2]) / rl;
      double w_angle = std::max(0.0, cosang);
      double wd = w_angle * wd_dir;
      // float32 implementations carry ~5e-7 absolute error in w_dir near the blend-zone edge
      if (std::fabs(wd - p.w_min) < 1e-6) bl = true;
      if (wd < p.w_min) {
        if (bl) B.border[l] = 1;
        continue;
      }
      running_average(B.sdf[l], B.w[l], dd, wd, p.w_max);
      B.sdf[l] = store_sdf(p, B.sdf[l], &bl);
      B.w[l] = store_w(p, B.w[l], &bl);
      n_upd++;
      if (p.with_color && rgb) {
        double dist = std::sqrt((pw[0] - x[0]) * (pw[0] - x[0]) + (pw[1] - x[1]) * (pw[1] - x[1]) +
                                (pw[2] - x[2]) * (pw[2] - x[2]));
        double wc = wd * (1.0 - std::min(1.0, dist / p.tau));  // eq. color_weight
        // the colour weight vanishes at |p - x| = tau; within 1e-6 of it a float32
        // implementation may round it to zero (no colour update) or keep a tiny weight
        if (std::fabs(1.0 - dist / p.tau) < 1e-6) bl = true;
        if (wc > 0.0) {
          for (int c = 0; c < 3; ++c) {
            double val = ((double)B.rgb[l][c] * B.wc[l] + (double)rgb[3 * pi + c] * wc) /
                         (B.wc[l] + wc);
            // colour is stored as 8-bit code: round half to even, as a quantised code both
            // implementations take in their own precision; ties within 1e-6 are borderline
            double fr = val - std::floor(val);
            if (std::fabs(fr - 0.5) < 1e-6) bl = true;
            double q = std::nearbyint(val);
            B.rgb[l][c] = (uint8_t)std::min(255.0, std::max(0.0, q));
          }
          B.wc[l] = store_w(p, std::min(B.wc[l] + wc, p.w_max), &bl);
        }
      }
      if (bl) B.border[l] = 1;
    }
  }
  s.updated = n_upd;
  s.carved = n_carve;
  if (st) *st = s;
}

// Export in ascending (bx, by, bz, D) order.  keys: n x 4 int32; sdf, w, wc: n x 512 float32
// (rounded from double); rgb: n x 512 x 3; border: n x 512.  Any output may be NULL.
int64_t orc_export(void* h, int32_t* keys, float* sdf, float* w, uint8_t* rgb, float* wc,
                   uint8_t* border) {
  Map& m = *static_cast<Map*>(h);
  std::vector<int> order(m.bricks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const Key& ka = m.keys[a];
    const Key& kb = m.keys[b];
    if (ka.x != kb.x) return ka.x < kb.x;
    if (ka.y != kb.y) return ka.y < kb.y;
    if (ka.z != kb.z) return ka.z < kb.z;
    return ka.d < kb.d;
  });
  for (size_t j = 0; j < order.size(); ++j) {
    const Brick& B = m.bricks[order[j]];
    const Key& k = m.keys[order[j]];
    if (keys) {
      keys[4 * j] = k.x;
      keys[4 * j + 1] = k.y;
      keys[4 * j + 2] = k.z;
      keys[4 * j + 3] = k.d;
    }
    for (int l = 0; l < kVox; ++l) {
      if (sdf) sdf[j * kVox + l] = (float)B.sdf[l];
      if (w) w[j * kVox + l] = (float)B.w[l];
      if (wc) wc[j * kVox + l] = (float)B.wc[l];
      if (rgb)
        for (int c = 0; c < 3; ++c) rgb[(j * kVox + l) * 3 + c] = B.rgb[l][c];
      if (border) border[j * kVox + l] = B.border[l];
    }
  }
  return (int64_t)order.size();
}

// Recycling (Sec. 3): every brick none of whose observed voxels (w > 0) holds a value below
// t_free -- free space after repeated carving, or never observed -- leaves the map.  Returns
// the number removed; the remaining bricks keep their contents and border flags.
int64_t orc_recycle(void* h, double t_free) {
  Map& m = *static_cast<Map*>(h);
  std::vector<Key> keys;
  std::deque<Brick> bricks;
  int64_t removed = 0;
  for (size_t i = 0; i < m.bricks.size(); ++i) {
    const Brick& B = m.bricks[i];
    bool surface = false;
    for (int l = 0; l < kVox && !surface; ++l) surface = B.w[l] > 0.0 && B.sdf[l] < t_free;
    if (!surface) {
      ++removed;
      continue;
    }
    keys.push_back(m.keys[i]);
    bricks.push_back(B);
  }
  m.keys.swap(keys);
  m.bricks.swap(bricks);
  m.index.clear();
  m.blocks.clear();
  for (size_t i = 0; i < m.keys.size(); ++i) {
    m.index.emplace(m.keys[i], (int)i);
    m.blocks.insert(BKey{m.keys[i].x, m.keys[i].y, m.keys[i].z});
  }
  return removed;
}

// Replace the map contents with n bricks (same layout as orc_export; rgb and wc may be NULL).
void orc_import(void* h, int64_t n, const int32_t* keys, const float* sdf, const float* w,
                const uint8_t* rgb, const float* wc) {
  Map& m = *static_cast<Map*>(h);
  m.index.clear();
  m.blocks.clear();
  m.keys.clear();
  m.bricks.clear();
  for (int64_t j = 0; j < n; ++j) {
    int id = add_brick(m, Key{keys[4 * j], keys[4 * j + 1], keys[4 * j + 2], keys[4 * j + 3]});
    Brick& B = m.bricks[id];
    for (int l = 0; l < kVox; ++l) {
      B.sdf[l] = sdf[j * kVox + l];
      B.w[l] = w[j * kVox + l];
      B.wc[l] = wc ? wc[j * kVox + l] : 0.0;
      for (int c = 0; c < 3; ++c) B.rgb[l][c] = rgb ? rgb[(j * kVox + l) * 3 + c] : 0;
    }
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Rendering (Sec. 4)
// ---------------------------------------------------------------------------------------

namespace {

struct DirSample {
  bool defined;
  double phi, W, grad[3], n[3];
  bool grad_ok;
  double omega;          // combination weight (gradient form or fallback, see eval)
  bool color_ok;
  double rgb[3], Wc;
};

struct Sample {
  bool defined;
  double f;
  bool fallback;          // gradient-weight sum was zero: eq. combine_tsdf_weight used
  double S_rel;           // gradient-weight sum / sum of W over defined directions
  DirSample dir[6];
  int touched[6][8];      // brick ordinals read (-1 none), for byte accounting
};

struct Tracker {
  std::vector<uint8_t>* geom;   // may be null
  const Map* m;
};

// Evaluates the combined SDF at world point x for unit ray direction r (Sec. 4).
//
// Per direction D: the trilinear interpolant of the eight corner voxels of the cell
// containing x gives Phi^D, W^D and (analytically) grad Phi^D; Phi^D is defined only if all
// eight corners are allocated in D and carry W > 0.  The combination weight is
// w_dir(n^D) * max(0, <n^D, -r>) * W^D(x) (eq. combine_weight; a negative cosine is clamped
// to zero), with n^D the normalised gradient (valid if |grad| * s >= 1e-6).  When these
// weights sum to zero over the defined directions, the weights W^D(x) * max(0, <v^D, -r>)
// of eq. combine_tsdf_weight are used.  f = sum(omega Phi) / sum(omega); undefined if no
// direction is defined or the weights still sum to zero.
//
// `margin` (0 for the definition itself) is added to every factor before it is clamped at
// zero; evaluating with +/- a small margin exposes samples whose branch depends on a factor
// sitting at its threshold (used only to classify grazing pixels).
Sample eval(const Map& m, const double x[3], const double r[3], std::vector<uint8_t>* touched,
            double margin = 0.0) {
  const Params& p = m.p;
  Sample S;
  S.defined = false;
  S.f = 0;
  S.fallback = false;
  S.S_rel = 0;
  for (int d = 0; d < 6; ++d)
    for (int c = 0; c < 8; ++c) S.touched[d][c] = -1;
  double vx[3], a[3];
  int64_t i0[3];
  for (int k = 0; k < 3; ++k) {
    vx[k] = x[k] / p.voxel;
    double fl = std::floor(vx[k]);
    i0[k] = (int64_t)fl;
    a[k] = vx[k] - fl;
  }
  if (m.blocks.find(BKey{(int32_t)floor_div(i0[0], kB), (int32_t)floor_div(i0[1], kB),
                         (int32_t)floor_div(i0[2], kB)}) == m.blocks.end()) {
    for (int d = 0; d < 6; ++d) S.dir[d].defined = false;
    return S;
  }
  double sumW = 0, sumO = 0, sumOP = 0;
  for (int d = 0; d < 6; ++d) {
    DirSample& ds = S.dir[d];
    ds.defined = false;
    ds.grad_ok = false;
    ds.color_ok = false;
    ds.omega = 0;
    ds.n[0] = ds.n[1] = ds.n[2] = 0.0;
    if (p.single_direction && d != 0) continue;
    double sd[8], ww[8], cc[8][3], wcc[8];
    bool ok = true, cok = true;
    for (int c = 0; c < 8 && ok; ++c) {
      int64_t v[3] = {i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + ((c >> 2) & 1)};
      int64_t b[3] = {floor_div(v[0], kB), floor_div(v[1], kB), floor_div(v[2], kB)};
      auto it = m.index.find(Key{(int32_t)b[0], (int32_t)b[1], (int32_t)b[2], d});
      if (it == m.index.end()) {
        ok = false;
        break;
      }
      S.touched[d][c] = it->second;
      const Brick& B = m.bricks[it->second];
      int l = (int)((v[0] - kB * b[0]) + kB * (v[1] - kB * b[1]) + kB * kB * (v[2] - kB * b[2]));
      sd[c] = B.sdf[l];
      ww[c] = B.w[l];
      if (!(ww[c] > 0.0)) ok = false;
      for (int ch = 0; ch < 3; ++ch) cc[c][ch] = B.rgb[l][ch];
      wcc[c] = B.wc[l];
      if (!(wcc[c] > 0.0)) cok = false;
    }
    if (touched)
      for (int c = 0; c < 8; ++c)
        if (S.touched[d][c] >= 0) (*touched)[S.touched[d][c]] = 1;
    if (!ok) continue;
    ds.defined = true;
    // trilinear weights of corner c = (cx, cy, cz)
    double tw[8];
    for (int c = 0; c < 8; ++c)
      tw[c] = ((c & 1) ? a[0] : 1 - a[0]) * (((c >> 1) & 1) ? a[1] : 1 - a[1]) *
              (((c >> 2) & 1) ? a[2] : 1 - a[2]);
    ds.phi = 0;
    ds.W = 0;
    for (int c = 0; c < 8; ++c) {
      ds.phi += tw[c] * sd[c];
      ds.W += tw[c] * ww[c];
    }
    // analytic gradient of the trilinear interpolant, per metre
    for (int k = 0; k < 3; ++k) {
      double g = 0;
      for (int c = 0; c < 8; ++c) {
        double wk = 1.0;
        for (int j = 0; j < 3; ++j) {
          if (j == k) continue;
          int bit = (c >> j) & 1;
          wk *= bit ? a[j] : 1 - a[j];
        }
        g += (((c >> k) & 1) ? 1.0 : -1.0) * wk * sd[c];
      }
      ds.grad[k] = g / p.voxel;
    }
    double gl = std::sqrt(dot3(ds.grad, ds.grad));
    ds.grad_ok = gl * p.voxel >= 1e-6;
    if (ds.grad_ok)
      for (int k = 0; k < 3; ++k) ds.n[k] = ds.grad[k] / gl;
    if (p.single_direction) {
      ds.omega = ds.W;    // regular TSDF: the one volume is used as is
    } else if (ds.grad_ok) {
      double mr[3] = {-r[0], -r[1], -r[2]};
      double wd = margin == 0.0 ? w_dir(p, ds.n, d) : w_dir_shifted(p, ds.n, d, margin);
      ds.omega = wd * std::max(0.0, dot3(ds.n, mr) + margin) * ds.W;
    }
    sumW += ds.W;
    if (cok && p.with_color) {
      ds.color_ok = true;
      ds.Wc = 0;
      for (int ch = 0; ch < 3; ++ch) ds.rgb[ch] = 0;
      for (int c = 0; c < 8; ++c) {
        ds.Wc += tw[c] * wcc[c];
        for (int ch = 0; ch < 3; ++ch) ds.rgb[ch] += tw[c] * cc[c][ch];
      }
    }
  }
  bool any = false;
  for (int d = 0; d < 6; ++d)
    if (S.dir[d].defined) {
      any = true;
      sumO += S.dir[d].omega;
      sumOP += S.dir[d].omega * S.dir[d].phi;
    }
  if (!any) return S;
  S.S_rel = sumW > 0 ? sumO / sumW : 0;
  if (sumO > 0.0) {
    S.defined = true;
    S.f = sumOP / sumO;
    return S;
  }
  // eq. combine_tsdf_weight: no direction offers a usable gradient weight
  S.fallback = true;
  sumO = 0;
  sumOP = 0;
  for (int d = 0; d < 6; ++d) {
    DirSample& ds = S.dir[d];
    if (!ds.defined) continue;
    double vr = -(kAxis[d][0] * r[0] + kAxis[d][1] * r[1] + kAxis[d][2] * r[2]);
    ds.omega = ds.W * std::max(0.0, vr + margin);
    sumO += ds.omega;
    sumOP += ds.omega * ds.phi;
  }
  if (sumO > 0.0) {
    S.defined = true;
    S.f = sumOP / sumO;
  }
  return S;
}

// Distance of x (voxel units) to the nearest cell face, minimum over the three axes.
double face_distance(const Map& m, const double x[3]) {
  double best = 1.0;
  for (int k = 0; k < 3; ++k) {
    double v = x[k] / m.p.voxel;
    double fr = v - std::floor(v);
    best = std::min(best, std::min(fr, 1.0 - fr));
  }
  return best;
}

// Shading outputs of a sample on the ray r (Sec. 4): the normal, normalised weighted sum of
// the per-direction gradient normals, or of the axis vectors on the fallback branch (the
// paper does not specify it), world frame, has_n false where the weights sum to zero; the
// colour, per direction the trilinear colour over corners with w_c > 0, blended with
// w_dir(n^D) max(0, <n^D, -r>) W_c^D(x), and where those sum to zero with the geometric
// combination weights (the paper does not specify how colours are combined), unrounded,
// has_c false where no weight is positive.
struct Shade {
  double n[3], rgb[3];
  bool has_n, has_c;
};

Shade shade(const Params& p, const Sample& S, const double r[3]) {
  Shade o{{0, 0, 0}, {0, 0, 0}, false, false};
  double nw[3] = {0, 0, 0};
  for (int d = 0; d < 6; ++d) {
    const DirSample& ds = S.dir[d];
    if (!ds.defined || ds.omega <= 0) continue;
    for (int k = 0; k < 3; ++k) nw[k] += ds.omega * (S.fallback ? kAxis[d][k] : ds.n[k]);
  }
  const double nl = std::sqrt(dot3(nw, nw));
  if (nl > 0) {
    o.has_n = true;
    for (int k = 0; k < 3; ++k) o.n[k] = nw[k] / nl;
  }
  if (!p.with_color) return o;
  double so = 0, sc[3] = {0, 0, 0};
  const double mr[3] = {-r[0], -r[1], -r[2]};
  for (int d = 0; d < 6; ++d) {
    const DirSample& ds = S.dir[d];
    if (!ds.defined || !ds.color_ok || !ds.grad_ok || S.fallback) continue;
    const double oc = w_dir(p, ds.n, d) * std::max(0.0, dot3(ds.n, mr)) * ds.Wc;
    so += oc;
    for (int ch = 0; ch < 3; ++ch) sc[ch] += oc * ds.rgb[ch];
  }
  if (!(so > 0)) {
    so = 0;
    sc[0] = sc[1] = sc[2] = 0;
    for (int d = 0; d < 6; ++d) {
      const DirSample& ds = S.dir[d];
      if (!ds.defined || !ds.color_ok) continue;
      so += ds.omega;
      for (int ch = 0; ch < 3; ++ch) sc[ch] += ds.omega * ds.rgb[ch];
    }
  }
  if (so > 0) {
    o.has_c = true;
    for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = sc[ch] / so;
  }
  return o;
}

}  // namespace

extern "C" {

// Grazing flags of a rendered pixel (bits of `flags`):
enum {
  kNearZero = 1,      // a lattice sample up to the hit has |f| < eps_f
  kNearFace = 2,      // a lattice sample up to the hit lies within eps_x (voxels) of a cell
                      // face and moving it by 2 eps_x across that face changes definedness or
                      // the sign test
  kBranch = 4,        // a lattice sample up to the hit changes definedness, branch (gradient
                      // weights or fallback) or sign when every thresholded factor is moved
                      // by +/- eps_s
  kAmbiguous = 8,     // the bracket holds more than one sign change (undefined points count
                      // as free space)
  kRootFace = 16,     // the root lies inside a cell but within eps_root metres of one of its
                      // faces: a refinement with that tolerance may take the outputs from
                      // the neighbouring cell (normal, colour)
  kRootBranch = 32,   // where normal and colour are taken, the combination switches branch
                      // (gradient weights or fallback) or definedness when the thresholded
                      // factors move by +/- eps_s, or within eps_root metres along the ray
  kRootShade = 64,    // the shading outputs are not fixed at the resolution eps_root of the
                      // root: eps_root metres beyond it along the ray the normal has turned by
                      // more than eps_n, a colour channel has moved by more than eps_c or the
                      // colour appears or vanishes (combination weights near zero change
                      // their ratio that fast)
};

struct OrcRenderCfg {
  double z_near, z_far;
  double eps_f, eps_x, eps_s, eps_root;
  int32_t classify;   // 0: skip the grazing classification (plain render)
  double eps_n;       // radians
  double eps_c;       // colour levels (0 .. 255)
};

// Renders pixels (us[i], vs[i]) of a camera with intrinsics (fx, fy, cx, cy) and pose T
// (camera to world).  Outputs per pixel (NULL allowed): depth, vertex (3, camera frame),
// normal (3, camera frame), rgba (4), mask, flags, hit lattice index k and refined t.
// touched_geom: optional per-brick byte array marked for every brick a sample read.
void orc_render(void* h, int64_t n, const int32_t* us, const int32_t* vs, double fx, double fy,
                double cx, double cy, const double T[16], const OrcRenderCfg* cfg, double* depth,
                double* vertex, double* normal, uint8_t* rgba, uint8_t* mask, uint8_t* flags,
                int64_t* khit, double* thit, uint8_t* touched_geom) {
  const Map& m = *static_cast<Map*>(h);
  const Params& p = m.p;
  double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  double c0[3] = {T[3], T[7], T[11]};
  std::vector<uint8_t> touched_all;
  if (touched_geom) touched_all.assign(m.bricks.size(), 0);

#pragma omp parallel
  {
    std::vector<uint8_t> touched_local;
    if (touched_geom) touched_local.assign(m.bricks.size(), 0);
    std::vector<uint8_t>* tl = touched_geom ? &touched_local : nullptr;
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
      int u = us[i], v = vs[i];
      double dc[3] = {(u - cx) / fx, (v - cy) / fy, 1.0};
      double len = std::sqrt(dot3(dc, dc));
      double rc[3] = {dc[0] / len, dc[1] / len, dc[2] / len};
      double r[3];
      for (int k = 0; k < 3; ++k) r[k] = R[3 * k] * rc[0] + R[3 * k + 1] * rc[1] + R[3 * k + 2] * rc[2];
      double t0 = cfg->z_near / rc[2], tmax = cfg->z_far / rc[2];
      uint8_t fl = 0;
      bool hit = false;
      int64_t kh = -1;
      bool prev_def = false;
      double prev_f = 0;
      double ta = 0, tb = 0;
      for (int64_t k = 0;; ++k) {
        double tk = t0 + (double)k * p.step;   // lattice point from its integer index
        if (tk > tmax) break;
        double x[3] = {c0[0] + tk * r[0], c0[1] + tk * r[1], c0[2] + tk * r[2]};
        Sample S = eval(m, x, r, tl);
        // grazing classification of this lattice sample
        if (cfg->classify && S.defined && std::fabs(S.f) < cfg->eps_f) fl |= kNearZero;
        if (cfg->classify) {
          bool any_def = false;
          for (int d = 0; d < 6; ++d) any_def |= S.dir[d].defined;
          if (any_def) {
            Sample lo = eval(m, x, r, nullptr, -cfg->eps_s);
            Sample hi = eval(m, x, r, nullptr, cfg->eps_s);
            if (lo.defined != hi.defined || lo.fallback != hi.fallback ||
                (lo.defined && (lo.f > 0) != (hi.f > 0)))
              fl |= kBranch;
          }
        }
        if (cfg->classify && face_distance(m, x) < cfg->eps_x) {
          bool pos = S.defined && S.f > 0, def = S.defined;
          for (int ax = 0; ax < 3; ++ax)
            for (int sg = -1; sg <= 1; sg += 2) {
              double y[3] = {x[0], x[1], x[2]};
              y[ax] += sg * 2.0 * cfg->eps_x * p.voxel;
              Sample S2 = eval(m, y, r, nullptr);
              if (S2.defined != def || (S2.defined && (S2.f > 0) != pos)) fl |= kNearFace;
            }
        }
        if (k >= 1 && S.defined && prev_def && prev_f > 0.0 && S.f <= 0.0) {
          hit = true;
          kh = k;
          ta = t0 + (double)(k - 1) * p.step;
          tb = tk;
          break;
        }
        prev_def = S.defined;
        prev_f = S.f;
      }
      double out_depth = 0, out_v[3] = {0, 0, 0}, out_n[3] = {0, 0, 0};
      uint8_t out_c[4] = {0, 0, 0, 0};
      double ts = 0;
      if (hit) {
        auto f_at = [&](double tt, bool* def) {
          double x[3] = {c0[0] + tt * r[0], c0[1] + tt * r[1], c0[2] + tt * r[2]};
          Sample S = eval(m, x, r, tl);
          *def = S.defined;
          return S.f;
        };
        // ambiguity: more than one sign change among 64 samples of the bracket, undefined
        // points counting as free space as in the refinement below (an undefined stretch
        // between the positive and the negative end leaves the root unique)
        if (cfg->classify) {
          // 64 even steps, plus both sides of every cell face the bracket crosses (f may
          // jump there, and a jump can open a stretch of the other sign narrower than the
          // steps)
          std::vector<double> tt;
          for (int j = 0; j <= 64; ++j) tt.push_back(ta + (tb - ta) * j / 64.0);
          for (int k = 0; k < 3; ++k) {
            if (r[k] == 0.0) continue;
            const double xa_ = (c0[k] + ta * r[k]) / p.voxel, xb_ = (c0[k] + tb * r[k]) / p.voxel;
            for (double fc = std::ceil(std::min(xa_, xb_)); fc <= std::max(xa_, xb_); fc += 1.0) {
              const double tf = (fc * p.voxel - c0[k]) / r[k];
              for (double dlt : {-1e-9, 1e-9})
                if (tf + dlt > ta && tf + dlt < tb) tt.push_back(tf + dlt);
            }
          }
          std::sort(tt.begin(), tt.end());
          int changes = 0;
          bool lastpos = true;
          for (size_t j = 0; j < tt.size(); ++j) {
            bool def;
            double fv = f_at(tt[j], &def);
            bool pos = !def || fv > 0;
            if (j > 0 && pos != lastpos) changes++;
            lastpos = pos;
          }
          if (changes > 1) fl |= kAmbiguous;
        }
        // refinement on the bracket (Sec. 4: small steps driven by the interpolated SDF):
        // bisection until the bracket is below 1e-9 m; undefined points count as free space
        double a = ta, b = tb;
        while (b - a > 1e-9) {
          double c = 0.5 * (a + b);
          bool def;
          double fc = f_at(c, &def);
          if (!def || fc > 0.0)
            a = c;
          else
            b = c;
        }
        ts = 0.5 * (a + b);
        // normal and colour are taken at the bracket end inside the surface (f <= 0, always
        // defined): where f jumps across a cell face this is the cell beyond the face
        double xs[3] = {c0[0] + b * r[0], c0[1] + b * r[1], c0[2] + b * r[2]};
        Sample S = eval(m, xs, r, tl);
        const Shade sh = shade(p, S, r);
        if (cfg->classify) {
          // a refinement to eps_root ends inside the surface, between the root and eps_root
          // beyond it
          {
            const double y[3] = {xs[0] + cfg->eps_root * r[0], xs[1] + cfg->eps_root * r[1],
                                 xs[2] + cfg->eps_root * r[2]};
            const Shade sy = shade(p, eval(m, y, r, nullptr), r);
            bool moved = sy.has_n != sh.has_n || sy.has_c != sh.has_c;
            if (sy.has_n && sh.has_n)
              moved |= std::acos(std::min(1.0, dot3(sy.n, sh.n))) > cfg->eps_n;
            if (sy.has_c && sh.has_c)
              for (int ch = 0; ch < 3; ++ch) moved |= std::fabs(sy.rgb[ch] - sh.rgb[ch]) > cfg->eps_c;
            if (moved) fl |= kRootShade;
          }
          const Sample lo = eval(m, xs, r, nullptr, -cfg->eps_s);
          const Sample hi = eval(m, xs, r, nullptr, cfg->eps_s);
          const double xf[3] = {xs[0] + cfg->eps_root * r[0], xs[1] + cfg->eps_root * r[1],
                                xs[2] + cfg->eps_root * r[2]};
          const Sample Sf = eval(m, xf, r, nullptr);
          if (lo.defined != hi.defined || lo.fallback != hi.fallback ||
              Sf.defined != S.defined || Sf.fallback != S.fallback)
            fl |= kRootBranch;
          double xa[3] = {c0[0] + a * r[0], c0[1] + a * r[1], c0[2] + a * r[2]};
          bool same_cell = true;
          for (int k = 0; k < 3; ++k)
            same_cell &= std::floor(xa[k] / p.voxel) == std::floor(xs[k] / p.voxel);
          if (same_cell) {
            double far[3], near_[3];
            for (int k = 0; k < 3; ++k) {
              far[k] = xs[k] + cfg->eps_root * r[k];
              near_[k] = xs[k] - cfg->eps_root * r[k];
            }
            for (int k = 0; k < 3; ++k)
              if (std::floor(far[k] / p.voxel) != std::floor(xs[k] / p.voxel) ||
                  std::floor(near_[k] / p.voxel) != std::floor(xs[k] / p.voxel))
                fl |= kRootFace;
          }
        }
        out_depth = ts * rc[2];
        for (int k = 0; k < 3; ++k) out_v[k] = ts * rc[k];
        if (sh.has_n)
          for (int k = 0; k < 3; ++k)  // world -> camera: R^T n
            out_n[k] = R[k] * sh.n[0] + R[3 + k] * sh.n[1] + R[6 + k] * sh.n[2];
        if (sh.has_c) {
          for (int ch = 0; ch < 3; ++ch)
            out_c[ch] = (uint8_t)std::min(255.0, std::max(0.0, std::nearbyint(sh.rgb[ch])));
          out_c[3] = 255;
        }
      }
      if (depth) depth[i] = out_depth;
      if (vertex)
        for (int k = 0; k < 3; ++k) vertex[3 * i + k] = out_v[k];
      if (normal)
        for (int k = 0; k < 3; ++k) normal[3 * i + k] = out_n[k];
      if (rgba)
        for (int k = 0; k < 4; ++k) rgba[4 * i + k] = out_c[k];
      if (mask) mask[i] = hit ? 1 : 0;
      if (flags) flags[i] = fl;
      if (khit) khit[i] = kh;
      if (thit) thit[i] = ts;
    }
    if (touched_geom) {
#pragma omp critical
      for (size_t j = 0; j < touched_local.size(); ++j) touched_all[j] |= touched_local[j];
    }
  }
  if (touched_geom)
    for (size_t j = 0; j < touched_all.size(); ++j) touched_geom[j] = touched_all[j];
}

// Evaluates the combined SDF at n world points (for pins of the definition): f, defined,
// fallback flag.
void orc_eval(void* h, int64_t n, const double* xs, const double* rs, double* f, uint8_t* def,
              uint8_t* fallback) {
  const Map& m = *static_cast<Map*>(h);
  for (int64_t i = 0; i < n; ++i) {
    Sample S = eval(m, xs + 3 * i, rs + 3 * i, nullptr);
    f[i] = S.f;
    def[i] = S.defined;
    fallback[i] = S.fallback;
  }
}

// Shading outputs (see shade) at world points xs (n, 3) for unit rays rs (n, 3): world-frame
// unit normal (zero where none), unrounded colour, and bit 0 / bit 1 of `has` for the normal
// / colour being present.
void orc_shade(void* h, int64_t n, const double* xs, const double* rs, double* normal,
               double* rgb, uint8_t* has) {
  const Map& m = *static_cast<Map*>(h);
  for (int64_t i = 0; i < n; ++i) {
    const Shade o = shade(m.p, eval(m, xs + 3 * i, rs + 3 * i, nullptr), rs + 3 * i);
    for (int k = 0; k < 3; ++k) {
      normal[3 * i + k] = o.n[k];
      rgb[3 * i + k] = o.rgb[k];
    }
    has[i] = (o.has_n ? 1 : 0) | (o.has_c ? 2 : 0);
  }
}

// Brick ordinal -> export position map is not needed: touched arrays use internal ordinals,
// so expose the key of an internal ordinal.
void orc_brick_key(void* h, int64_t id, int32_t* key4) {
  const Map& m = *static_cast<Map*>(h);
  const Key& k = m.keys[(size_t)id];
  key4[0] = k.x;
  key4[1] = k.y;
  key4[2] = k.z;
  key4[3] = k.d;
}

double orc_w_dir(const Params* p, const double n[3], int d) { return w_dir(*p, n, d); }

// Threads an OpenMP region of the oracle uses.
int orc_num_threads() { return omp_get_max_threads(); }

}  // extern "C"

// ---------------------------------------------------------------------------------------
// View-dependent combined ("rendering") TSDF (Sec. 4: Lemma positional_unambiguity, the
// precomputed combined TSDF, conditional recombination; Sec. 7: evaluation at integer voxel
// positions with six-neighbour gradients)
// ---------------------------------------------------------------------------------------

namespace {

struct Frustum {
  double R[9], t[3];                // camera -> world of the frustum's pose
  double fx, fy, cx, cy;
  double umin, umax, vmin, vmax;    // accepted projections: [umin, umax) x [vmin, vmax)
};

Frustum make_frustum(const double T[16], int W, int H, double fx, double fy, double cx,
                     double cy, double margin) {
  Frustum F;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) F.R[3 * r + c] = T[4 * r + c];
    F.t[r] = T[4 * r + 3];
  }
  F.fx = fx;
  F.fy = fy;
  F.cx = cx;
  F.cy = cy;
  // pixel centres sit at integer coordinates, so the image covers [-1/2, W - 1/2); it is
  // widened by `margin` times its size on every side
  F.umin = -0.5 - margin * W;
  F.umax = W - 0.5 + margin * W;
  F.vmin = -0.5 - margin * H;
  F.vmax = H - 0.5 + margin * H;
  return F;
}

// Whether world point x lies in front of the camera and projects into the widened image.
// `edge` receives how close the decision is: the distance in pixels to the nearest bound, or
// |z| in metres when z is within 1e-9 m of zero.
bool in_frustum(const Frustum& F, const double x[3], double* edge) {
  double d[3] = {x[0] - F.t[0], x[1] - F.t[1], x[2] - F.t[2]};
  double y[3];
  for (int k = 0; k < 3; ++k) y[k] = F.R[k] * d[0] + F.R[3 + k] * d[1] + F.R[6 + k] * d[2];
  if (std::fabs(y[2]) < 1e-9) {
    *edge = 0.0;
    return false;
  }
  if (y[2] < 0.0) {
    *edge = 1e30;
    return false;
  }
  double u = F.fx * y[0] / y[2] + F.cx, v = F.fy * y[1] / y[2] + F.cy;
  *edge = std::min(std::min(std::fabs(u - F.umin), std::fabs(u - F.umax)),
                   std::min(std::fabs(v - F.vmin), std::fabs(v - F.vmax)));
  return u >= F.umin && u < F.umax && v >= F.vmin && v < F.vmax;
}

// Brick of direction d holding voxel v (world voxel index), and the voxel's local index.
const Brick* brick_at(const Map& m, const int64_t v[3], int d, int* l) {
  int64_t b[3] = {floor_div(v[0], kB), floor_div(v[1], kB), floor_div(v[2], kB)};
  auto it = m.index.find(Key{(int32_t)b[0], (int32_t)b[1], (int32_t)b[2], d});
  if (it == m.index.end()) return nullptr;
  *l = (int)((v[0] - kB * b[0]) + kB * (v[1] - kB * b[1]) + kB * kB * (v[2] - kB * b[2]));
  return &m.bricks[it->second];
}

struct Combined {
  bool defined;
  double f;
  bool fallback;
  double S_rel;        // gradient-weight sum / sum of W over the observed directions
  bool color;
  bool color_blend;    // the colour came from the w_dir max(0, <n, -r>) W_c blend
  double rgb[3];
};

// Combined SDF of the six directions at voxel v for a camera centred at c (eq.
// combine_weight at the voxel centre x = v s, view ray r = (x - c) / |x - c|).  Direction D
// takes part if the voxel is observed in it (W^D > 0); its normal n^D is the normalised
// central difference of Phi^D over the six axis neighbours, usable only if all six are
// observed in D and |grad| s >= 1e-6.  Weights w_dir(n^D) max(0, <n^D, -r>) W^D; when these
// sum to zero, eq. combine_tsdf_weight over the observed directions.  Colour: the voxel
// colours of the directions on the gradient branch blended with w_dir(n^D) max(0, <n^D, -r>)
// W_c^D (directions with W_c^D > 0), else with the combination weights; undefined if those
// sum to zero.  `margin` is added to every thresholded factor (classification only).
Combined combine_voxel(const Map& m, const int64_t v[3], const double c[3], double margin) {
  const Params& p = m.p;
  Combined C;
  C.defined = false;
  C.f = 0.0;
  C.fallback = false;
  C.S_rel = 0.0;
  C.color = false;
  C.color_blend = false;
  C.rgb[0] = C.rgb[1] = C.rgb[2] = 0.0;
  double x[3] = {v[0] * p.voxel, v[1] * p.voxel, v[2] * p.voxel};
  double r[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  double rl = std::sqrt(dot3(r, r));
  if (!(rl > 0.0)) return C;
  for (int k = 0; k < 3; ++k) r[k] /= rl;
  const double mr[3] = {-r[0], -r[1], -r[2]};
  bool obs[6] = {false, false, false, false, false, false}, gok[6] = {false, false, false, false, false, false};
  double phi[6], W[6], n[6][3], om[6], rgb[6][3], Wc[6];
  double sumW = 0, sumO = 0, sumOP = 0;
  for (int d = 0; d < 6; ++d) {
    om[d] = 0.0;
    int l;
    const Brick* B = brick_at(m, v, d, &l);
    if (!B || !(B->w[l] > 0.0)) continue;
    obs[d] = true;
    phi[d] = B->sdf[l];
    W[d] = B->w[l];
    Wc[d] = B->wc[l];
    for (int ch = 0; ch < 3; ++ch) rgb[d][ch] = B->rgb[l][ch];
    double g[3];
    bool all = true;
    for (int k = 0; k < 3 && all; ++k) {
      int64_t vp[3] = {v[0], v[1], v[2]}, vm[3] = {v[0], v[1], v[2]};
      vp[k] += 1;
      vm[k] -= 1;
      int lp, lm;
      const Brick* Bp = brick_at(m, vp, d, &lp);
      const Brick* Bm = brick_at(m, vm, d, &lm);
      if (!Bp || !Bm || !(Bp->w[lp] > 0.0) || !(Bm->w[lm] > 0.0)) {
        all = false;
        break;
      }
      g[k] = (Bp->sdf[lp] - Bm->sdf[lm]) / (2.0 * p.voxel);
    }
    if (all) {
      double gl = std::sqrt(dot3(g, g));
      gok[d] = gl * p.voxel >= 1e-6;
      if (gok[d])
        for (int k = 0; k < 3; ++k) n[d][k] = g[k] / gl;
    }
    if (gok[d]) {
      double wd = margin == 0.0 ? w_dir(p, n[d], d) : w_dir_shifted(p, n[d], d, margin);
      om[d] = wd * std::max(0.0, dot3(n[d], mr) + margin) * W[d];
    }
    sumW += W[d];
    sumO += om[d];
    sumOP += om[d] * phi[d];
  }
  if (!(sumW > 0.0)) return C;
  C.S_rel = sumO / sumW;
  if (sumO > 0.0) {
    C.defined = true;
    C.f = sumOP / sumO;
  } else {
    // eq. combine_tsdf_weight
    C.fallback = true;
    sumO = sumOP = 0.0;
    for (int d = 0; d < 6; ++d) {
      if (!obs[d]) continue;
      om[d] = W[d] * std::max(0.0, dot3(kAxis[d], mr) + margin);
      sumO += om[d];
      sumOP += om[d] * phi[d];
    }
    if (sumO > 0.0) {
      C.defined = true;
      C.f = sumOP / sumO;
    }
  }
  if (!C.defined || !p.with_color) return C;
  double so = 0, sc[3] = {0, 0, 0};
  if (!C.fallback)
    for (int d = 0; d < 6; ++d) {
      if (!obs[d] || !gok[d] || !(Wc[d] > 0.0)) continue;
      double wd = margin == 0.0 ? w_dir(p, n[d], d) : w_dir_shifted(p, n[d], d, margin);
      double oc = wd * std::max(0.0, dot3(n[d], mr) + margin) * Wc[d];
      so += oc;
      for (int ch = 0; ch < 3; ++ch) sc[ch] += oc * rgb[d][ch];
    }
  C.color_blend = so > 0.0;
  if (!(so > 0.0)) {
    so = 0;
    sc[0] = sc[1] = sc[2] = 0;
    for (int d = 0; d < 6; ++d) {
      if (!obs[d] || !(Wc[d] > 0.0)) continue;
      so += om[d];
      for (int ch = 0; ch < 3; ++ch) sc[ch] += om[d] * rgb[d][ch];
    }
  }
  if (so > 0.0) {
    C.color = true;
    for (int ch = 0; ch < 3; ++ch) C.rgb[ch] = sc[ch] / so;
  }
  return C;
}

// Whether the discrete outcomes of combine_voxel (defined, branch, colour defined and its
// blend, the gradient test) could change under rounding: they differ between margins of +/- eps, a
// gradient length lies within 0.1 % of its threshold, or the gradient weights are tiny next
// to the observed weights (S_rel < 1e-3: every eligible direction is at a grazing or
// blend-zone edge, where f is ill-conditioned).
bool combine_fragile(const Map& m, const int64_t v[3], const double c[3], double eps,
                     const Combined& C0) {
  Combined a = combine_voxel(m, v, c, eps), b = combine_voxel(m, v, c, -eps);
  if (a.defined != C0.defined || b.defined != C0.defined || a.fallback != C0.fallback ||
      b.fallback != C0.fallback || a.color != C0.color || b.color != C0.color ||
      a.color_blend != C0.color_blend || b.color_blend != C0.color_blend)
    return true;
  if (C0.defined && !C0.fallback && C0.S_rel < 1e-3) return true;
  for (int d = 0; d < 6; ++d) {
    double g[3];
    bool all = true;
    for (int k = 0; k < 3 && all; ++k) {
      int64_t vp[3] = {v[0], v[1], v[2]}, vm[3] = {v[0], v[1], v[2]};
      vp[k] += 1;
      vm[k] -= 1;
      int lp, lm;
      const Brick* Bp = brick_at(m, vp, d, &lp);
      const Brick* Bm = brick_at(m, vm, d, &lm);
      if (!Bp || !Bm || !(Bp->w[lp] > 0.0) || !(Bm->w[lm] > 0.0)) {
        all = false;
        break;
      }
      g[k] = (Bp->sdf[lp] - Bm->sdf[lm]) / (2.0 * m.p.voxel);
    }
    if (all && std::fabs(std::sqrt(dot3(g, g)) * m.p.voxel / 1e-6 - 1.0) < 1e-3) return true;
  }
  return false;
}

}  // namespace

extern "C" {

// Combined TSDF of map `src` written into map `dst` (a single-direction map: direction 0
// holds the combined value, weight 1 where defined and 0 where not, the colour code and
// colour weight 1 where a colour is defined).  Every block of src gets its dst brick.
//   only_missing == 0 (recombination): every voxel centre inside the frustum of T_frustum
//     (image widened by margin_frac of its size per side) gets its combined value for the
//     camera centre of T_center; every other voxel holds no value.
//   only_missing != 0 (voxels seen for the first time): only voxels inside that frustum that
//     hold no value are evaluated; the others keep theirs.
// dst's border byte of a voxel: bit 0 the frustum decision is within eps_edge pixels
// (1e-9 m in depth) of its bound, bit 1 combine_fragile with margin eps_s.
void orc_combine(void* hsrc, void* hdst, const double Tc[16], const double Tf[16], int W, int H,
                 double fx, double fy, double cx, double cy, double margin_frac,
                 int only_missing, double eps_s, double eps_edge) {
  const Map& src = *static_cast<Map*>(hsrc);
  Map& dst = *static_cast<Map*>(hdst);
  const Frustum F = make_frustum(Tf, W, H, fx, fy, cx, cy, margin_frac);
  const double c[3] = {Tc[3], Tc[7], Tc[11]};
  std::vector<BKey> blocks(src.blocks.begin(), src.blocks.end());
  std::vector<int> ids(blocks.size());
  for (size_t i = 0; i < blocks.size(); ++i)
    ids[i] = add_brick(dst, Key{blocks[i].x, blocks[i].y, blocks[i].z, 0});
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < (int64_t)blocks.size(); ++i) {
    Brick& B = dst.bricks[ids[i]];
    for (int l = 0; l < kVox; ++l) {
      int64_t v[3] = {(int64_t)blocks[i].x * kB + (l % kB), (int64_t)blocks[i].y * kB + (l / kB) % kB,
                      (int64_t)blocks[i].z * kB + l / (kB * kB)};
      double x[3] = {v[0] * src.p.voxel, v[1] * src.p.voxel, v[2] * src.p.voxel};
      double edge;
      bool inside = in_frustum(F, x, &edge);
      if (only_missing && (B.w[l] > 0.0 || !inside)) continue;
      uint8_t flags = edge < eps_edge ? 1 : 0;
      if (!inside) {
        B.sdf[l] = 0.0;
        B.w[l] = 0.0;
        B.wc[l] = 0.0;
        B.rgb[l][0] = B.rgb[l][1] = B.rgb[l][2] = 0;
        B.border[l] = flags;
        continue;
      }
      Combined C = combine_voxel(src, v, c, 0.0);
      if (combine_fragile(src, v, c, eps_s, C)) flags |= 2;
      B.sdf[l] = C.defined ? C.f : 0.0;
      B.w[l] = C.defined ? 1.0 : 0.0;
      B.wc[l] = C.color ? 1.0 : 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        // stored as 8-bit codes, rounded half to even
        double q = C.color ? std::nearbyint(C.rgb[ch]) : 0.0;
        B.rgb[l][ch] = (uint8_t)std::min(255.0, std::max(0.0, q));
      }
      B.border[l] = flags;
    }
  }
}

}  // extern "C"
