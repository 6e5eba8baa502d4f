// Ray-cast rendering of the Directional TSDF (Sec. 4).
//
// One thread per pixel; a workgroup is one wave covering a work tile of 64 pixels (a single
// view's or a small batch's taken as 2x2 quads interleaved over a 128x32 pixel region, see
// tile_pixel; a large batch's an 8x8 tile).  Tiles are numbered so that the workgroups the dispatcher
// sends to one XCD (workgroup id mod 8) cover one contiguous band of the image, keeping each
// band's bricks in that XCD's L2.  Per ray:
//   * lattice t_k = t0 + k * step from z_near to z_far (Sec. 4: probing at regular intervals);
//     sample positions are float64 so that the cell a sample falls in is the exact one,
//     interpolation and combination are float32;
//   * blocks are found through the dense render index.  A sample whose base voxel lies in an
//     absent block is undefined in every direction, so the march jumps to the first lattice
//     point past the largest empty cell (64, 16 or 4 cm at 5 mm voxels) of the occupancy
//     hierarchy that contains the block.  In a sub-block whose skip bit is set every value a
//     cell based there can interpolate is positive, so the combined SDF is positive wherever
//     defined and no crossing can end there: only its last lattice point is evaluated (it may
//     start a crossing in what follows).  Both jumps are exact;
//   * per present direction: trilinear Phi^D, W^D and the analytic gradient of the interpolant
//     over the 8 corners (all corners allocated with W > 0, else the direction is undefined);
//     combination weight w_dir(n^D) max(0, <n^D, -r>) W^D (eq. combine_weight) and the
//     gradient-free fallback W^D max(0, <v^D, -r>) (eq. combine_tsdf_weight), both summed in
//     one pass over the directions;
//   * hit: first k >= 1 with f(t_{k-1}) > 0 >= f(t_k), both defined; the bracket is refined
//     to 1e-6 m (Newton or Illinois regula falsi steps, probes next to cell faces where f
//     may jump, bisections; see kRefineTol), undefined points counting as free space; outputs
//     are evaluated at the bracket end inside the surface.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dtsdf_internal.hpp"

using namespace dtsdf;

namespace {

struct RenderArgs {
  int W, H;
  int tiles_x, tiles;     // 8x8 pixel tiles (the batched launch)
  int itiles_x, itiles;   // interleaved work tiles (the single-view launch, see tile_pixel)
  int ilv;                // batched launch: this view's work tiles are interleaved
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
  int32_t* trace_counts;
  int help;       // lanes whose ray has finished evaluate points of the marching rays
};

// Work tiles of the single-view launch.  A wave renders 64 pixels of one work tile, as 16
// quads of 2x2 pixels.  The work tiles of a group of kIlvX x kIlvY take interleaved quads of
// the group's (8 kIlvX) x (8 kIlvY) pixel region (quad (qx, qy) of tile (tx, ty) is quad
// column kIlvX qx + tx mod kIlvX and row kIlvY qy + ty mod kIlvY of the region), so that the
// rays of a slow image region (grazing a surface, along a silhouette) are spread over many
// waves instead of holding one wave while the rest of the chip idles.  Interleaving makes a
// wave's rays less coherent (more distinct blocks per pass; the quads keep four neighbouring
// rays together), which costs total work; it pays only where the launch is bound by its
// slowest waves.  A batched launch therefore interleaves only while its work is small (up to
// kIlvBatchTiles 8x8 tiles, about three rounds of resident waves: one request's pyramid at up
// to 848x480) and otherwise, its views overlapping their tails, keeps plain 8x8 tiles.  The
// tile grid is padded to whole groups; lanes whose pixel lies outside the image start
// finished.
constexpr int kIlvX = 16, kIlvY = 4;
constexpr int64_t kIlvBatchTiles = 9000;

struct Trace {
  uint8_t* bricks;
  uint8_t* color;
  uint8_t* slots;
};

// Ray parameter at which the ray leaves the box [lo, hi) (world units).
__device__ inline double box_exit(const double o[3], const double ir[3], const double lo[3],
                                  const double hi[3]) {
  double t = 1e300;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (ir[ax] > 0.0) t = fmin(t, (hi[ax] - o[ax]) * ir[ax]);
    else if (ir[ax] < 0.0) t = fmin(t, (lo[ax] - o[ax]) * ir[ax]);
  }
  return t;
}

// Parameter of the first voxel face (a plane x = j * voxel on any axis) the ray crosses after t.
__device__ inline double face_after(const double o[3], const double r[3], const double ir[3],
                                    double t, double voxel, double inv_voxel) {
  double best = 1e300;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (r[ax] == 0.0) continue;
    const double x = (o[ax] + t * r[ax]) * inv_voxel;
    const double pl = (r[ax] > 0.0 ? floor(x) + 1.0 : ceil(x) - 1.0) * voxel;
    best = fmin(best, (pl - o[ax]) * ir[ax]);
  }
  return best;
}

__device__ inline void tile_pixel(const RenderArgs& a, int tile, int lane, int& u, int& v) {
  const int tx = tile % a.itiles_x, ty = tile / a.itiles_x;
  const int dx = lane & 1, dy = (lane >> 1) & 1, qx = (lane >> 2) & 3, qy = lane >> 4;
  u = (tx / kIlvX) * (8 * kIlvX) + 2 * (kIlvX * qx + tx % kIlvX) + dx;
  v = (ty / kIlvY) * (8 * kIlvY) + 2 * (kIlvY * qy + ty % kIlvY) + dy;
}

__device__ inline int64_t grid_index(const MapView& m, int bx, int by, int bz) {
  const int ix = bx - m.gx0, iy = by - m.gy0, iz = bz - m.gz0;
  if (ix < 0 || iy < 0 || iz < 0 || ix >= m.gx || iy >= m.gy || iz >= m.gz) return -1;
  return ((int64_t)iz * m.gy + iy) * m.gx + ix;
}

// Enters grid block `gi` (-1: outside the grid): its record, positive-cell words and group
// bytes are loaded in one round of independent loads (an absent block's words are read too
// and ignored, so that no load waits for the record) and kept in the lane's LDS columns:
// brick indices of direction d at row[d * 64], cell word z at cw[z * 64], group word w at
// gw[w * 64].  Returns the record's info word (0 outside the grid) and the present-direction
// mask in `pm`.  Bit kRecInGrid of the returned word marks a block inside the grid.
constexpr uint32_t kRecInGrid = 1u << 16;
template <bool TRACE>
__device__ inline uint32_t enter_block(const MapView& m, int64_t gi, int* row, uint64_t* cw,
                                       uint64_t* gw, uint32_t& pm, const Trace& tr) {
  pm = 0;
  if (gi < 0) {
#pragma unroll
    for (int d = 0; d < 6; ++d) row[d * 64] = -1;
    return 0;
  }
  const uint4* rp = reinterpret_cast<const uint4*>(m.grid_rec + gi);
  const uint4* cp = reinterpret_cast<const uint4*>(m.grid_cell + (size_t)gi * 8);
  const uint4* gp = reinterpret_cast<const uint4*>(m.grid_group + (size_t)gi * 64);
  const uint4 r0 = rp[0], r1 = rp[1];
  uint4 q[4], qg[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    q[h] = cp[h];
    qg[h] = gp[h];
  }
  const int b[6] = {(int)r0.x, (int)r0.y, (int)r0.z, (int)r0.w, (int)r1.x, (int)r1.y};
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    row[d * 64] = b[d];
    pm |= b[d] >= 0 ? 1u << d : 0u;
  }
  if (TRACE && tr.slots && (int)r1.w >= 0) tr.slots[(int)r1.w] = 1;
  if (r1.z & kRecPresent) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      cw[(2 * h) * 64] = (uint64_t)q[h].x | ((uint64_t)q[h].y << 32);
      cw[(2 * h + 1) * 64] = (uint64_t)q[h].z | ((uint64_t)q[h].w << 32);
      gw[(2 * h) * 64] = (uint64_t)qg[h].x | ((uint64_t)qg[h].y << 32);
      gw[(2 * h + 1) * 64] = (uint64_t)qg[h].z | ((uint64_t)qg[h].w << 32);
    }
  }
  return r1.z | kRecInGrid;
}

struct CellPos {
  int bl[3], lo[3];
  float a[3];
};

__device__ inline void locate(const MapView& m, const double x[3], CellPos& c) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vx = x[k] * m.inv_voxel;
    const double fl = floor(vx);
    const int ix = (int)fl;
    c.a[k] = (float)(vx - fl);
    c.bl[k] = ix >> 3;
    c.lo[k] = ix & 7;
  }
}

// arccos by the polynomial of Abramowitz & Stegun 4.4.46 (|error| <= 2e-8 on [0, 1]),
// extended to [-1, 0) by acos(x) = pi - acos(-x).
__device__ inline float acos_as(float x) {
  const float ax = fminf(fabsf(x), 1.0f);
  float p = -0.0012624911f;
  p = fmaf(p, ax, 0.0066700901f);
  p = fmaf(p, ax, -0.0170881256f);
  p = fmaf(p, ax, 0.0308918810f);
  p = fmaf(p, ax, -0.0501743046f);
  p = fmaf(p, ax, 0.0889789874f);
  p = fmaf(p, ax, -0.2145988016f);
  p = fmaf(p, ax, 1.5707963050f);
  const float r = sqrtf(1.0f - ax) * p;
  return x < 0.f ? 3.14159265358979f - r : r;
}

// Direction weight of Sec. 3 (clamped-linear reading), from the cosine <n, v^D>.
__device__ inline float w_dir_fast(float c, float theta, float inv_band) {
  return fminf(1.0f, fmaxf(0.0f, (theta - acos_as(c)) * inv_band));
}

struct Eval {
  bool defined;
  bool fallback;
  float f;
  float n[3];       // FULL: sum of omega * (n^D or v^D)
  float rgb[3];     // FULL: combined colour
  bool color_ok;
};

// Raw voxel word of the (sdf, w) field as it sits in memory: float2 in the plain layout, one
// 32-bit code word in the packed layouts (decoded only when used, so that a group of
// directions keeps half the registers in flight).
template <int F>
struct GeoRaw {
  using T = uint32_t;
  __device__ static void decode(T v, float& s, float& w) { Vox<F>::decode(v, s, w); }
};
template <>
struct GeoRaw<0> {
  using T = float2;
  __device__ static void decode(T v, float& s, float& w) {
    s = v.x;
    w = v.y;
  }
};
template <>
struct GeoRaw<kRegularVolume> : GeoRaw<0> {};

// Combined SDF (and, FULL, normal and colour) in the cell `cp` whose base block has bricks
// `brow` (grid records for the neighbour blocks at the cell's +x/+y/+z faces).  Directions are taken per lane in ascending order of D, so every lane pays only for
// the directions allocated in its own block.  They are processed in groups of G: the
// neighbour-brick lookups of a whole group are issued together, then the 8 G corner loads,
// and only then is any of them used, so that a group costs one chain of dependent loads
// instead of one per direction.  The sums are accumulated in ascending D, as one direction
// at a time would, so the result does not depend on G.
// NP points of one cell are evaluated together: point 0 at cp, point j > 0 at the
// fractional position pa[j - 1] of the same cell; the corner values are loaded once.
template <int F, bool FULL, bool TRACE, int NP, int G>
__device__ void eval_cell(const MapView& m, const CellPos& cp, uint32_t pm, const int* brow,
                          const float r[3], float inv_band, Eval* ev, const Trace& tr,
                          const float (*pa)[3] = nullptr) {
  static_assert(NP == 1 || !FULL, "outputs are evaluated one point at a time");
  // a regular volume: one value per voxel, weight 1, so f is the interpolant itself, the
  // normal its gradient and the colour its colour
  constexpr bool REG = F == kRegularVolume;
  using Raw = typename GeoRaw<F>::T;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    ev[j].defined = false;
    ev[j].fallback = false;
    ev[j].f = 0.f;
  }
  Eval& e = ev[0];
  if (FULL) {
    e.n[0] = e.n[1] = e.n[2] = 0.f;
    e.rgb[0] = e.rgb[1] = e.rgb[2] = 0.f;
    e.color_ok = false;
  }
  if (pm == 0) return;
  const int lx = cp.lo[0], ly = cp.lo[1], lz = cp.lo[2];
  // corners leaving the base block: x when lx == 7, y when ly == 7, z when lz == 7
  const int need = (lx == 7 ? 1 : 0) | (ly == 7 ? 2 : 0) | (lz == 7 ? 4 : 0);
  // grid indices of the blocks at offset o (o & need == o), else -1; their records are read
  // per direction below, every load issued unconditionally (absent ones read record 0) so
  // that they overlap instead of queueing behind one another
  int64_t ns[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) ns[o] = -1;
  if (need) {
#pragma unroll
    for (int o = 1; o < 8; ++o) {
      const int64_t gi = grid_index(m, cp.bl[0] + (o & 1), cp.bl[1] + ((o >> 1) & 1),
                                    cp.bl[2] + ((o >> 2) & 1));
      ns[o] = (o & need) == o ? gi : -1;
      if (TRACE && tr.slots && ns[o] >= 0 && m.grid_rec[ns[o]].slot >= 0)
        tr.slots[m.grid_rec[ns[o]].slot] = 1;
    }
  }
  const float ax = cp.a[0], ay = cp.a[1], az = cp.a[2];
  const float bx = 1.f - ax, by = 1.f - ay, bz = 1.f - az;
  const float tw[8] = {bx * by * bz, ax * by * bz, bx * ay * bz, ax * ay * bz,
                       bx * by * az, ax * by * az, bx * ay * az, ax * ay * az};
  // further points: combination sums of each (the first point's sums are so .. fop)
  float so2[NP > 1 ? NP - 1 : 1], sop2[NP > 1 ? NP - 1 : 1], fo2[NP > 1 ? NP - 1 : 1],
      fop2[NP > 1 ? NP - 1 : 1];
#pragma unroll
  for (int j = 0; j + 1 < NP; ++j) so2[j] = sop2[j] = fo2[j] = fop2[j] = 0.f;
  const float mr[3] = {-r[0], -r[1], -r[2]};
  // offsets of the four corner rows (y, z), (y + 1, z), (y, z + 1), (y + 1, z + 1) within
  // their bricks
  const int y1 = (ly + 1) & 7, z1 = (lz + 1) & 7;
  const uint32_t rq[4] = {(uint32_t)(8 * ly + 64 * lz), (uint32_t)(8 * y1 + 64 * lz),
                          (uint32_t)(8 * ly + 64 * z1), (uint32_t)(8 * y1 + 64 * z1)};
  const bool xin = lx < 7;
  float so = 0.f, sop = 0.f;   // gradient combination weights
  float fo = 0.f, fop = 0.f;   // fallback weights
  bool any = false;
  float ng0 = 0.f, ng1 = 0.f, ng2 = 0.f, nf0 = 0.f, nf1 = 0.f, nf2 = 0.f;
  float cg0 = 0.f, cg1 = 0.f, cg2 = 0.f, cgo = 0.f;     // colour weights of the colour blend
  float cgg0 = 0.f, cgg1 = 0.f, cgg2 = 0.f, cggo = 0.f; // geometric weights, gradient branch
  float cgf0 = 0.f, cgf1 = 0.f, cgf2 = 0.f, cgfo = 0.f; // geometric weights, fallback branch
  while (pm) {
    // ---- the next G present directions, ascending --------------------------------------
    int dg[G];
    bool ok[G];
    int br[G][8];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ok[g] = pm != 0;
      dg[g] = ok[g] ? __builtin_ctz(pm) : 0;
      pm &= pm - 1;
      const int b0 = brow[dg[g] * 64];
#pragma unroll
      for (int c = 0; c < 8; ++c) br[g][c] = b0;
    }
    if (need) {
      // corner c lies in the block at offset c & need; the lookups of the whole group are
      // issued before any is used
      int nbr[G][8];
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int o = 1; o < 8; ++o) {
          const int64_t so_ = ns[o];
          const int bo = m.grid_rec[so_ >= 0 ? so_ : 0].brick[dg[g]];
          nbr[g][o] = so_ >= 0 ? bo : -1;
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int o = 1; o < 8; ++o) {
          if ((o & need) != o) continue;
#pragma unroll
          for (int c = 1; c < 8; ++c)
            if ((c & o) == o) br[g][c] = (c & need) == o ? nbr[g][o] : br[g][c];
        }
#pragma unroll
        for (int c = 1; c < 8; ++c) ok[g] = ok[g] && br[g][c] >= 0;
      }
    }
    // ---- all corner loads of the group --------------------------------------------------
    // corner 2q at x = lx and corner 2q + 1 at x = lx + 1 of row q (x = 0 of the brick at +x
    // when lx == 7); a direction that is not evaluated reads voxel 0 of brick 0 instead
    Raw raw[G][8];
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t ia = (uint32_t)br[g][2 * q] * kVox + rq[q] + (uint32_t)lx;
        const uint32_t ib = xin ? ia + 1u : (uint32_t)br[g][2 * q + 1] * kVox + rq[q];
        raw[g][2 * q] = static_cast<const Raw*>(m.geo)[ok[g] ? ia : 0u];
        raw[g][2 * q + 1] = static_cast<const Raw*>(m.geo)[ok[g] ? ib : 0u];
        if (TRACE && tr.bricks && ok[g]) {
          tr.bricks[br[g][2 * q]] = 1;
          tr.bricks[br[g][2 * q + 1]] = 1;
        }
      }
    }
    // ---- contributions, in ascending D ----------------------------------------------
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!ok[g]) continue;
      const int d = dg[g];
      float sv[8], wv[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) GeoRaw<F>::decode(raw[g][c], sv[c], wv[c]);
      // defined only if every corner has W > 0; evaluated regardless (then dropped by
      // zero weights) so that the distance loads need not wait for the weight test
      bool wok = true;
#pragma unroll
      for (int c = 0; c < 8; ++c) wok = wok && (wv[c] > 0.f);
      any = any || wok;
      float phi = 0.f, W = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        phi = fmaf(tw[c], sv[c], phi);
        W = fmaf(tw[c], wv[c], W);
      }
      // analytic gradient of the interpolant (per voxel)
      const float gx = (sv[1] - sv[0]) * by * bz + (sv[3] - sv[2]) * ay * bz +
                       (sv[5] - sv[4]) * by * az + (sv[7] - sv[6]) * ay * az;
      const float gy = (sv[2] - sv[0]) * bx * bz + (sv[3] - sv[1]) * ax * bz +
                       (sv[6] - sv[4]) * bx * az + (sv[7] - sv[5]) * ax * az;
      const float gz = (sv[4] - sv[0]) * bx * by + (sv[5] - sv[1]) * ax * by +
                       (sv[6] - sv[2]) * bx * ay + (sv[7] - sv[3]) * ax * ay;
      const float gl = sqrtf(gx * gx + gy * gy + gz * gz);
      float om = 0.f, wdc = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
      if (REG) {
        if (gl >= 1e-6f) {
          const float il = 1.f / gl;
          n0 = gx * il;
          n1 = gy * il;
          n2 = gz * il;
        }
        wdc = 1.f;
        om = 1.f;
      } else if (gl >= 1e-6f) {
        const float il = 1.f / gl;
        n0 = gx * il;
        n1 = gy * il;
        n2 = gz * il;
        const float wd = w_dir_fast(axis_dot(n0, n1, n2, d), m.theta, inv_band);
        wdc = wd * fmaxf(0.f, n0 * mr[0] + n1 * mr[1] + n2 * mr[2]);
        om = wdc * W;
      }
      om = wok ? om : 0.f;
      wdc = wok ? wdc : 0.f;
      so += om;
      sop += om * phi;
      const float fb = wok ? W * fmaxf(0.f, axis_dot(mr[0], mr[1], mr[2], d)) : 0.f;
      fo += fb;
      fop += fb * phi;
#pragma unroll
      for (int j = 0; j + 1 < NP; ++j) {
        const float px = pa[j][0], py = pa[j][1], pz = pa[j][2];
        const float qx = 1.f - px, qy = 1.f - py, qz = 1.f - pz;
        const float uw[8] = {qx * qy * qz, px * qy * qz, qx * py * qz, px * py * qz,
                             qx * qy * pz, px * qy * pz, qx * py * pz, px * py * pz};
        float phj = 0.f, Wj = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          phj = fmaf(uw[c], sv[c], phj);
          Wj = fmaf(uw[c], wv[c], Wj);
        }
        const float hx = (sv[1] - sv[0]) * qy * qz + (sv[3] - sv[2]) * py * qz +
                         (sv[5] - sv[4]) * qy * pz + (sv[7] - sv[6]) * py * pz;
        const float hy = (sv[2] - sv[0]) * qx * qz + (sv[3] - sv[1]) * px * qz +
                         (sv[6] - sv[4]) * qx * pz + (sv[7] - sv[5]) * px * pz;
        const float hz = (sv[4] - sv[0]) * qx * qy + (sv[5] - sv[1]) * px * qy +
                         (sv[6] - sv[2]) * qx * py + (sv[7] - sv[3]) * px * py;
        const float hl = sqrtf(hx * hx + hy * hy + hz * hz);
        float omj = 0.f;
        if (REG) {
          omj = 1.f;
        } else if (hl >= 1e-6f) {
          const float il = 1.f / hl;
          const float m0 = hx * il, m1 = hy * il, m2 = hz * il;
          const float wd = w_dir_fast(axis_dot(m0, m1, m2, d), m.theta, inv_band);
          omj = wd * fmaxf(0.f, m0 * mr[0] + m1 * mr[1] + m2 * mr[2]) * Wj;
        }
        omj = wok ? omj : 0.f;
        so2[j] += omj;
        sop2[j] += omj * phj;
        const float fbj = wok ? Wj * fmaxf(0.f, axis_dot(mr[0], mr[1], mr[2], d)) : 0.f;
        fo2[j] += fbj;
        fop2[j] += fbj * phj;
      }
      if (FULL) {
        ng0 += om * n0;
        ng1 += om * n1;
        ng2 += om * n2;
        const float sfb = (d & 1) ? -fb : fb;
        nf0 += d < 2 ? sfb : 0.f;
        nf1 += (d >> 1) == 1 ? sfb : 0.f;
        nf2 += d >= 4 ? sfb : 0.f;
        if (m.with_color && wok) {
          float wsum = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
          bool cok = true;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int loc = ((lx + (c & 1)) & 7) + 8 * ((ly + ((c >> 1) & 1)) & 7) +
                            64 * ((lz + ((c >> 2) & 1)) & 7);
            const size_t vi = (size_t)br[g][c] * kVox + loc;
            if (TRACE && tr.color) tr.color[br[g][c]] = 1;
            float w;
            uint32_t code;
            Vox<F>::load_color(m.rgb, m.wc, vi, code, w);
            cok = cok && (w > 0.f);
            wsum = fmaf(tw[c], w, wsum);
            c0 = fmaf(tw[c], (float)(code & 0xFFu), c0);
            c1 = fmaf(tw[c], (float)((code >> 8) & 0xFFu), c1);
            c2 = fmaf(tw[c], (float)((code >> 16) & 0xFFu), c2);
          }
          if (cok) {
            const float oc = wdc * wsum;   // w_dir(n^D) max(0, <n^D, -r>) W_c^D
            cg0 += oc * c0;
            cg1 += oc * c1;
            cg2 += oc * c2;
            cgg0 += om * c0;
            cgg1 += om * c1;
            cgg2 += om * c2;
            cgf0 += fb * c0;
            cgf1 += fb * c1;
            cgf2 += fb * c2;
            cgo += oc;
            cggo += om;
            cgfo += fb;
          }
        }
      }
    }
  }
  if (!any) return;
  if (so > 0.f) {
    e.defined = true;
    e.f = sop / so;
  } else {
    // no usable gradient weight in any direction: eq. combine_tsdf_weight
    e.fallback = true;
    if (fo > 0.f) {
      e.defined = true;
      e.f = fop / fo;
    }
  }
#pragma unroll
  for (int j = 0; j + 1 < NP; ++j) {
    Eval& ej = ev[j + 1];
    if (so2[j] > 0.f) {
      ej.defined = true;
      ej.f = sop2[j] / so2[j];
    } else {
      ej.fallback = true;
      if (fo2[j] > 0.f) {
        ej.defined = true;
        ej.f = fop2[j] / fo2[j];
      }
    }
  }
  if (FULL) {
    e.n[0] = e.fallback ? nf0 : ng0;
    e.n[1] = e.fallback ? nf1 : ng1;
    e.n[2] = e.fallback ? nf2 : ng2;
    if (m.with_color) {
      float s0 = cg0, s1 = cg1, s2 = cg2, sw = cgo;
      if (e.fallback) {
        s0 = cgf0; s1 = cgf1; s2 = cgf2; sw = cgfo;
      } else if (!(cgo > 0.f)) {
        s0 = cgg0; s1 = cgg1; s2 = cgg2; sw = cggo;
      }
      if (sw > 0.f) {
        e.color_ok = true;
        const float isw = 1.f / sw;
        e.rgb[0] = s0 * isw;
        e.rgb[1] = s1 * isw;
        e.rgb[2] = s2 * isw;
      }
    }
  }
}

// Directions per group of the march's evaluations (see eval_cell).
constexpr int march_group(int) { return 1; }

// World-frame unit ray of pixel (u, v) of view `a` and its parameter range [t0, tmax] (depth
// z_near .. z_far).
__device__ inline void pixel_ray(const RenderArgs& a, int u, int v, double r[3], double& t0,
                                 double& tmax) {
  const double dc[3] = {((double)u - a.cx) / a.fx, ((double)v - a.cy) / a.fy, 1.0};
  const double len = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
  const double rc[3] = {dc[0] / len, dc[1] / len, dc[2] / len};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    r[k] = a.R[3 * k] * rc[0] + a.R[3 * k + 1] * rc[1] + a.R[3 * k + 2] * rc[2];
  t0 = a.z_near / rc[2];
  tmax = a.z_far / rc[2];
}

// Lane number of the n-th set bit (n counted from 0) of a 64-bit lane mask.
__device__ inline int nth_lane(uint64_t mask, int n) {
  int base = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t lo = mask & ((1ull << w) - 1ull);
    const int c = __popcll(lo);
    if (n >= c) {
      n -= c;
      mask >>= w;
      base += w;
    } else {
      mask = lo;
    }
  }
  return base;
}

__device__ inline double shfl_d(double x, int src) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __shfl((int)(b & 0xffffffff), src, 64);
  const int hi = __shfl((int)(b >> 32), src, 64);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Lattice points a marching ray may be helped with per pass (lanes whose own ray has finished
// evaluate them).
constexpr int kMaxHelpers = 7;

// Refinement of the bracket of a crossing, until it is shorter than kRefineTol (metres along
// the ray) or after kRefineMaxIter steps.  A step evaluates a pair of points kRefinePair on
// either side of an estimate (the pair is the final bracket when it straddles the root): the
// Newton step from the slope of the previous pair when that lands within a quarter of the
// bracket of it, else Illinois regula falsi.  Every fourth step, and after a step that shrank
// the bracket by less than a tenth, the step probes next to the first voxel face inside the
// bracket instead (f may jump where the cell changes: false position then stays pinned to
// one end), and bisects when no face lies inside.
constexpr double kRefineTol = 1e-6;
constexpr double kRefinePair = 0.45 * kRefineTol;
constexpr int kRefineMaxIter = 24;

// Renders pixel (u, v) of view `a`; every lane of the wave calls it (lanes outside the image
// pass inside = false and write nothing).
//
// Each pass of the outer loop evaluates the combined SDF once per lane.  Before it, every
// lane advances on its own through the cheap steps (jumps over absent space, positive
// sub-blocks and positive cells, refinement bookkeeping) until it holds its next evaluation
// point, so that the lanes of a wave evaluate together instead of taking turns.  A lattice
// point whose successor lies in the same cell is evaluated together with it (the corner
// values are loaded once), so a ray crossing the band at a grazing angle needs about half
// the passes.
template <int F, bool TRACE, int G>
__device__ void render_pixel(const MapView& m, const RenderArgs& a, int u, int v, bool inside) {
  const size_t i = (size_t)v * a.W + u;
  const size_t HW = (size_t)a.W * a.H;
  const float inv_band = 1.0f / (2.0f * m.theta - 1.5707963267948966f);
  double r[3];
  double t0, tmax;
  pixel_ray(a, u, v, r, t0, tmax);
  float rf[3] = {(float)r[0], (float)r[1], (float)r[2]};
  const double o[3] = {a.t[0], a.t[1], a.t[2]};
  const double step = m.step;
  const Trace tr{a.trace_bricks, a.trace_color, a.trace_slots};
  int n_eval = 0, n_skip = 0, n_absent = 0, n_refine = 0;
  const double ir[3] = {r[0] != 0.0 ? 1.0 / r[0] : 0.0, r[1] != 0.0 ? 1.0 / r[1] : 0.0,
                        r[2] != 0.0 ? 1.0 / r[2] : 0.0};
  const double inv_step = 1.0 / step;
  const double bw = kB * m.voxel;          // block edge [m]
  int cb0 = 0x7fffffff, cb1 = 0, cb2 = 0;  // block of the cached record
  // per lane (column `lane`): brick indices of the current block, direction d at row d;
  // its positive-cell words, slice z at row z; its group bytes, bytes 8 w .. 8 w + 7 at row w
  __shared__ int brick_rows[6 * 64];
  __shared__ uint64_t cell_words[8 * 64];
  __shared__ uint64_t group_words[8 * 64];
  const int lane = (int)(threadIdx.x & 63);
  int* const brow = brick_rows + lane;
  uint64_t* const cwl = cell_words + lane;
  uint64_t* const gwl = group_words + lane;
  uint32_t cpm = 0;               // present directions of the current block
  uint32_t cinfo = 0;             // record info word of the current block (see enter_block)
  int pos_last = -1;              // last lattice point of the current positive run
  bool prev_def = false, hit = false, refining = false, done = !inside;
  float prev_f = 0.f, fa = 0.f, fb = 0.f;
  double ta = 0.0, tb = 0.0;
  int k = 0;
  int it = 0, side = 0;
  bool bisect = false;    // refinement: the next step is a bisection (or a face probe)
  bool probe = false;     // refinement: the pending point is a face probe
  double tn = -1.0;       // refinement: Newton estimate from the last pair (-1: none)
  bool pending = false;   // te holds an evaluation point not evaluated yet
  double te = 0.0;        // parameter of the pending point
  double te2 = 0.0;       // second point evaluated with it (refinement pair, or lattice k + 1)
  bool lattice = false;   // the pending point is lattice point k, not a deferred one
  bool lpair = false;     // lattice: k + 1 is evaluated together with k
  int next_k = 0;         // lattice index after the pending point
  bool h_def = false;     // value of the point this lane evaluated in the current pass
  float h_f = 0.f;
  for (;;) {
    // ---- advance to the next evaluation point ---------------------------------------
    for (; !pending && !done;) {
      if (refining) {
        if (it >= kRefineMaxIter || !((tb - ta) > kRefineTol)) {
          done = true;
          break;
        }
        probe = false;
        if ((it & 3) != 3 && !bisect) {
          // false position, or the Newton step of the last pair when it stays well inside
          double tc = ta + (tb - ta) * (double)__fdividef(fa, fa - fb);
          if (tn > ta && tn < tb) tc = tn;
          if (!(tc > ta && tc < tb)) tc = 0.5 * (ta + tb);
          // the estimate is evaluated as a pair straddling it by kRefinePair: when the
          // estimate is that close to the root the pair is the final bracket
          te = fmax(tc - kRefinePair, 0.5 * (ta + tc));
          te2 = fmin(tc + kRefinePair, 0.5 * (tc + tb));
        } else {
          // f may jump where the cell changes: probe next to the first voxel face inside the
          // bracket (just before it, or just after it once the bracket starts there); with
          // no face inside, bisect
          const double tf = face_after(o, r, ir, ta, m.voxel, m.inv_voxel);
          if (tf < tb) {
            probe = true;
            te = tf - ta > 2.0 * kRefinePair ? tf - kRefinePair
                                             : fmin(tf + kRefinePair, 0.5 * (tf + tb));
            te2 = te;
          } else {
            const double tc = 0.5 * (ta + tb);
            te = fmax(tc - kRefinePair, 0.5 * (ta + tc));
            te2 = fmin(tc + kRefinePair, 0.5 * (tc + tb));
          }
        }
        pending = true;
        break;
      }
      const double tk = t0 + (double)k * step;
      if (tk > tmax) {
        done = true;
        break;
      }
      const double x[3] = {o[0] + tk * r[0], o[1] + tk * r[1], o[2] + tk * r[2]};
      CellPos cp;
      locate(m, x, cp);
      if (cp.bl[0] != cb0 || cp.bl[1] != cb1 || cp.bl[2] != cb2) {
        cb0 = cp.bl[0];
        cb1 = cp.bl[1];
        cb2 = cp.bl[2];
        cinfo = enter_block<TRACE>(m, grid_index(m, cb0, cb1, cb2), brow, cwl, gwl, cpm, tr);
      }
      if (!(cinfo & kRecPresent)) {
        const int gg[3] = {m.gx0, m.gy0, m.gz0};
        double texit;
        if (cinfo & kRecInGrid) {
          // absent block: leave the largest aligned empty cell containing it
          const int sh = (int)((cinfo >> 8) & 7u);   // log2 of its edge in blocks
          const int g[3] = {cb0 - m.gx0, cb1 - m.gy0, cb2 - m.gz0};
          double lo[3], hi[3];
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            const int c0 = gg[ax] + ((g[ax] >> sh) << sh);
            lo[ax] = (double)c0 * bw;
            hi[ax] = (double)(c0 + (1 << sh)) * bw;
          }
          texit = box_exit(o, ir, lo, hi);
        } else {
          // outside the index grid (which holds every block): go to where the ray enters
          // the grid box, or finish if it never does
          const int gd[3] = {m.gx, m.gy, m.gz};
          double tn = -1e300, tf = 1e300;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            const double lo = (double)gg[ax] * bw, hi = (double)(gg[ax] + gd[ax]) * bw;
            if (ir[ax] != 0.0) {
              const double t1 = (lo - o[ax]) * ir[ax], t2 = (hi - o[ax]) * ir[ax];
              tn = fmax(tn, fmin(t1, t2));
              tf = fmin(tf, fmax(t1, t2));
            } else if (o[ax] < lo || o[ax] >= hi) {
              tn = 1e300;
            }
          }
          texit = (tn < tf && tf > tk) ? tn : 1e300;
        }
        const double jn = ceil((texit - 1e-6 - t0) * inv_step);
        const int j0 = (int)fmin(jn, 1073741824.0);
        if (TRACE) ++n_absent;
        prev_def = false;
        pos_last = -1;
        k = j0 > k + 1 ? j0 : k + 1;
        continue;
      }
      const int sub = (cp.lo[0] >> 2) | ((cp.lo[1] >> 2) << 1) | ((cp.lo[2] >> 2) << 2);
      const bool pos_sub = (cinfo >> sub) & 1u;
      bool pos_cell = pos_sub;
      int ext = 4;   // edge of the positive box in cells: 4 (sub-block), 2 (cell group), 1
      if (!pos_sub) {
        // the cell, and the aligned 2x2x2 group of cells holding it (both slices of the pair)
        const uint64_t w0 = cwl[(cp.lo[2] & 6) * 64], w1 = cwl[((cp.lo[2] & 6) + 1) * 64];
        const uint64_t wc = (cp.lo[2] & 1) ? w1 : w0;
        pos_cell = (wc >> (cp.lo[0] + 8 * cp.lo[1])) & 1ull;
        const int gs = (cp.lo[0] & 6) + 8 * (cp.lo[1] & 6);
        ext = (((w0 & w1) >> gs) & 0x303ull) == 0x303ull ? 2 : 1;
      }
      if (pos_cell) {
        // positive sub-block, cell group or cell: no crossing can end in it; jump to its
        // last lattice point (evaluated only if the point after it is)
        double lo[3], hi[3];
        const int cbv[3] = {cb0, cb1, cb2};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int v0 = cbv[ax] * kB + (cp.lo[ax] & ~(ext - 1));
          lo[ax] = (double)v0 * m.voxel;
          hi[ax] = (double)(v0 + ext) * m.voxel;
        }
        const double texit = box_exit(o, ir, lo, hi);
        const double jn = ceil((texit - 1e-6 - t0) * inv_step);
        const int j0 = (int)fmin(jn, 1073741824.0);
        const int last = j0 - 1 > k ? j0 - 1 : k;
        if (t0 + (double)last * step > tmax) {
          done = true;
          break;
        }
        pos_last = last;
        k = last + 1;
        continue;
      }
      lpair = false;
      if (pos_last == k - 1 && k >= 1) {
        // the crossing test at k needs the value at k - 1, skipped so far
        te = t0 + (double)(k - 1) * step;
        lattice = false;
        next_k = k;
        pos_last = -1;
        if (TRACE) ++n_skip;
      } else {
        te = tk;
        lattice = true;
        next_k = k + 1;
        // lattice point k + 1 in the same cell: evaluated in the same pass
        te2 = t0 + (double)(k + 1) * step;
        if (te2 <= tmax) {
          const double x2[3] = {o[0] + te2 * r[0], o[1] + te2 * r[1], o[2] + te2 * r[2]};
          CellPos cp2;
          locate(m, x2, cp2);
          lpair = cp2.bl[0] == cp.bl[0] && cp2.bl[1] == cp.bl[1] && cp2.bl[2] == cp.bl[2] &&
                  cp2.lo[0] == cp.lo[0] && cp2.lo[1] == cp.lo[1] && cp2.lo[2] == cp.lo[2];
        }
        if (TRACE) n_eval += lpair ? 2 : 1;
      }
      pending = true;
    }
    // ---- evaluate -----------------------------------------------------------------
    if (!__any(pending)) break;
    // Lanes whose ray has finished help the marching rays: each takes one lattice point after
    // the ones its ray evaluates itself this pass.  The ray receives the values in order and
    // runs the crossing test over them as if it had evaluated them itself (f at a lattice
    // point does not depend on who evaluates it, and the points a march skips cannot end a
    // crossing), so the hit, and everything after it, is the same.  Owner and helper
    // exchange data by shuffles only; a helper's own ray keeps its bracket, and its
    // direction is recomputed for the outputs.
    const bool owner = pending && !refining;
    const uint64_t own_m = __ballot(owner);
    const uint64_t idle_m = __ballot(!pending);
    const int n_own = __popcll(own_m), n_idle = __popcll(idle_m);
    const int nh = (!TRACE && a.help && n_own > 0) ? min(kMaxHelpers, n_idle / n_own) : 0;
    const uint64_t below = (1ull << (threadIdx.x & 63)) - 1ull;
    // lattice index after the owner's own points: k (+ 1 with the pair), or k after a
    // deferred k - 1
    const int base = lattice ? (lpair ? k + 2 : k + 1) : next_k;
    int h_src = (int)(threadIdx.x & 63);
    bool helper = false;
    int h_k = 0;
    double h_tmax = 0.0;
    if (nh > 0) {
      int slot = -1;
      if (!pending) {
        const int hr = __popcll(idle_m & below);
        if (hr < nh * n_own) {
          slot = hr / n_own;
          h_src = nth_lane(own_m, hr % n_own);
        }
      }
      // every lane takes part in the shuffles (a lane that is no helper reads itself)
      double hr3[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) hr3[q] = shfl_d(r[q], h_src);
      const double h_t0 = shfl_d(t0, h_src);
      h_tmax = shfl_d(tmax, h_src);
      const int h_base = __shfl(base, h_src, 64);
      if (slot >= 0) {
        h_k = h_base + slot;
        const double th = h_t0 + (double)h_k * step;
        helper = th <= h_tmax;
        if (helper) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            r[q] = hr3[q];
            rf[q] = (float)hr3[q];
          }
          te = th;
        }
      }
    }
    if (pending || helper) {
      const double x[3] = {o[0] + te * r[0], o[1] + te * r[1], o[2] + te * r[2]};
      CellPos cp;
      locate(m, x, cp);
      if (cp.bl[0] != cb0 || cp.bl[1] != cb1 || cp.bl[2] != cb2) {
        cb0 = cp.bl[0];
        cb1 = cp.bl[1];
        cb2 = cp.bl[2];
        cinfo = enter_block<TRACE>(m, grid_index(m, cb0, cb1, cb2), brow, cwl, gwl, cpm, tr);
      }
      // a second point is evaluated with the first when both share the cell: the refinement
      // pair, or lattice point k + 1
      bool pair = pending && lattice && lpair;
      float pa1[1][3] = {{cp.a[0], cp.a[1], cp.a[2]}};
      if (pending && (refining || pair)) {
        const double x2[3] = {o[0] + te2 * r[0], o[1] + te2 * r[1], o[2] + te2 * r[2]};
        CellPos cp2;
        locate(m, x2, cp2);
        pair = cp2.bl[0] == cp.bl[0] && cp2.bl[1] == cp.bl[1] && cp2.bl[2] == cp.bl[2] &&
               cp2.lo[0] == cp.lo[0] && cp2.lo[1] == cp.lo[1] && cp2.lo[2] == cp.lo[2];
        pa1[0][0] = cp2.a[0];
        pa1[0][1] = cp2.a[1];
        pa1[0][2] = cp2.a[2];
      }
      Eval ev[2];
      // only the directions defined somewhere in the cell's 2x2x2 group can contribute
      const int grp = (cp.lo[0] >> 1) + 4 * (cp.lo[1] >> 1) + 16 * (cp.lo[2] >> 1);
      const uint32_t gdef = (uint32_t)(gwl[(grp >> 3) * 64] >> (8 * (grp & 7))) & 0x3Fu;
      eval_cell<F, false, TRACE, 2, G>(m, cp, cpm & gdef, brow, rf, inv_band, ev, tr, pa1);
      const Eval& e = ev[0];
      h_def = e.defined;
      h_f = e.f;
      if (pending) {
        pending = false;
        if (refining) {
          if (TRACE) ++n_refine;
          ++it;
          const double w0 = tb - ta;
          const bool pos1 = !e.defined || e.f > 0.f;
          const bool pos2 = !ev[1].defined || ev[1].f > 0.f;
          if (pos1 && pair && !pos2) {
            // the pair straddles the root: final bracket
            ta = te;
            tb = te2;
            if (e.defined) fa = e.f;
            fb = ev[1].f;
          } else if (pos1) {
            ta = pair ? te2 : te;
            const Eval& ea = pair ? ev[1] : e;
            if (ea.defined) fa = ea.f;
            if (side == 1) fb *= 0.5f;
            side = 1;
          } else {
            tb = te;
            fb = e.f;
            if (side == -1) fa *= 0.5f;
            side = -1;
          }
          // a step that shrank the bracket by less than a tenth (one end keeps a value far
          // from the root, e.g. behind a jump of f at a cell face), or a face probe that
          // leaves a face inside the bracket, is followed by a face probe or bisection
          bisect = (tb - ta) > 0.9 * w0 ||
                   (probe && face_after(o, r, ir, ta, m.voxel, m.inv_voxel) < tb);
          // Newton step from the pair's slope, kept when it lands within a quarter of the
          // bracket of the pair
          tn = -1.0;
          if (pair && e.defined && ev[1].defined && te2 > te) {
            const double sl = (double)(ev[1].f - e.f) / (te2 - te);
            if (sl < 0.0) {
              const double t_n = te - (double)e.f / sl;
              if (fabs(t_n - te) < 0.25 * (tb - ta)) tn = t_n;
            }
          }
        } else if (lattice && k >= 1 && e.defined && prev_def && prev_f > 0.f && e.f <= 0.f) {
          hit = true;
          refining = true;
          ta = t0 + (double)(k - 1) * step;
          tb = te;
          fa = prev_f;
          fb = e.f;
        } else if (pair) {
          // lattice point k + 1, with f(k) from the first point
          if (ev[1].defined && e.defined && e.f > 0.f && ev[1].f <= 0.f) {
            hit = true;
            refining = true;
            ta = te;
            tb = te2;
            fa = e.f;
            fb = ev[1].f;
          } else {
            prev_def = ev[1].defined;
            prev_f = ev[1].f;
            k = next_k + 1;
          }
        } else {
          prev_def = e.defined;
          prev_f = e.f;
          k = next_k;
        }
      }
    }
    // the helpers' values, in lattice order, for each marching ray that has not hit
    if (nh > 0) {
      const int my_rank = __popcll(own_m & below);
      bool take = owner && !refining && k == base;
      for (int sl = 0; sl < nh; ++sl) {
        const int hr = my_rank + sl * n_own;
        const int src = (owner && hr < n_idle) ? nth_lane(idle_m, hr) : (int)(threadIdx.x & 63);
        const int hv = __shfl(helper ? 1 : 0, src, 64);
        const int hd = __shfl(h_def ? 1 : 0, src, 64);
        const float hfv = __shfl(h_f, src, 64);
        take = take && owner && hr < n_idle && hv != 0;
        if (take) {
          pos_last = -1;
          if (k >= 1 && hd && prev_def && prev_f > 0.f && hfv <= 0.f) {
            hit = true;
            refining = true;
            ta = t0 + (double)(k - 1) * step;
            tb = t0 + (double)k * step;
            fa = prev_f;
            fb = hfv;
            take = false;
          } else {
            prev_def = hd != 0;
            prev_f = hfv;
            ++k;
          }
        }
      }
    }
  }
  float out_depth = 0.f, out_v[3] = {0.f, 0.f, 0.f}, out_n[3] = {0.f, 0.f, 0.f};
  uint32_t out_c = 0;
  if (hit) {
    pixel_ray(a, u, v, r, t0, tmax);
#pragma unroll
    for (int q = 0; q < 3; ++q) rf[q] = (float)r[q];
    const double ts = 0.5 * (ta + tb);
    const double x[3] = {o[0] + tb * r[0], o[1] + tb * r[1], o[2] + tb * r[2]};
    CellPos cp;
    locate(m, x, cp);
    uint32_t pm = 0;
    enter_block<TRACE>(m, grid_index(m, cp.bl[0], cp.bl[1], cp.bl[2]), brow, cwl, gwl, pm, tr);
    Eval e;
    eval_cell<F, true, TRACE, 1, 1>(m, cp, pm, brow, rf, inv_band, &e, tr);
    // the camera-frame ray again (not kept live through the march)
    const double dc[3] = {((double)u - a.cx) / a.fx, ((double)v - a.cy) / a.fy, 1.0};
    const double len = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    const double rc[3] = {dc[0] / len, dc[1] / len, dc[2] / len};
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
  if (!inside) return;
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
  if (TRACE && a.trace_counts) {
    a.trace_counts[4 * i + 0] = n_eval;
    a.trace_counts[4 * i + 1] = n_skip;
    a.trace_counts[4 * i + 2] = n_absent;
    a.trace_counts[4 * i + 3] = n_refine;
  }
}

// Three waves per SIMD (at most 168 VGPRs): the march is latency-bound and needs the waves.
template <int F, bool TRACE, int G = march_group(F)>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void render_k(
    MapView m, RenderArgs a) {
  // XCD-aware tile order: workgroup j runs on XCD j % 8; give each XCD a contiguous band
  const int per = (a.itiles + 7) >> 3;
  const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tile >= a.itiles) return;
  int u, v;
  tile_pixel(a, tile, (int)(threadIdx.x & 63), u, v);
  render_pixel<F, TRACE, G>(m, a, u, v, u < a.W && v < a.H);
}

// Views of different sizes in one persistent launch: every wave takes the next (view, tile)
// work item from a counter until all are done.  Each pixel is computed exactly as by
// render_k, so a view's output does not depend on the batch it is rendered in.
template <int F, bool TRACE, int G = march_group(F)>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void render_batch_k(MapView m, const RenderArgs* __restrict__ reqs,
                                                     const int32_t* __restrict__ prefix, int n,
                                                     int total, int32_t* counter) {
  for (;;) {
    int item = 0;
    if (threadIdx.x == 0) item = atomicAdd(counter, 1);
    item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
    if (item >= total) break;
    int lo = 0, hi = n;   // prefix[lo] <= item < prefix[lo + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (prefix[mid] <= item) lo = mid;
      else hi = mid;
    }
    const RenderArgs& a = reqs[lo];
    const int tile = item - prefix[lo];
    int u, v;
    if (a.ilv) {
      tile_pixel(a, tile, (int)(threadIdx.x & 63), u, v);
    } else {
      u = (tile % a.tiles_x) * 8 + (int)(threadIdx.x & 7);
      v = (tile / a.tiles_x) * 8 + (int)(threadIdx.x >> 3);
    }
    render_pixel<F, TRACE, G>(m, a, u, v, u < a.W && v < a.H);
  }
}

bool fill_args(const dtsdf_intrinsics* intr, const double T[16], float z_near, float z_far,
               const dtsdf_render_out* out, RenderArgs& a) {
  if (!intr || !T || !out || intr->width <= 0 || intr->height <= 0 || intr->width > 16384 ||
      intr->height > 16384 || !(intr->fx > 0) || !(intr->fy > 0) || !(z_near > 0) ||
      !(z_far > z_near))
    return false;
  if (out->rgba && ((uintptr_t)out->rgba & 3u)) return false;
  if (out->flags & ~DTSDF_RENDER_ALONE) return false;
  a.W = intr->width;
  a.H = intr->height;
  a.tiles_x = (a.W + 7) / 8;
  a.tiles = a.tiles_x * ((a.H + 7) / 8);
  // interleaved work tiles, padded to whole groups
  a.itiles_x = (a.tiles_x + kIlvX - 1) / kIlvX * kIlvX;
  a.itiles = a.itiles_x * (((a.H + 7) / 8 + kIlvY - 1) / kIlvY * kIlvY);
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
  a.trace_counts = out->trace_counts;
  a.help = (out->flags & DTSDF_RENDER_ALONE) ? 0 : 1;
  a.ilv = 0;
  return true;
}

}  // namespace

extern "C" dtsdf_status dtsdf_render(const dtsdf_map* m, const dtsdf_intrinsics* intr,
                                     const double T[16], float z_near, float z_far,
                                     const dtsdf_render_out* out, void* stream) {
  RenderArgs a;
  if (!m || !fill_args(intr, T, z_near, z_far, out, a)) return DTSDF_E_INVAL;
  const int per = (a.itiles + 7) / 8;
  const dim3 grd(per * 8);
  const bool trace = a.trace_bricks || a.trace_color || a.trace_slots || a.trace_counts;
  const MapView v = make_view(m);
  hipStream_t st = (hipStream_t)stream;
  if (m->regular) {
    if (trace) hipLaunchKernelGGL((render_k<kRegularVolume, true>), grd, dim3(64), 0, st, v, a);
    else hipLaunchKernelGGL((render_k<kRegularVolume, false>), grd, dim3(64), 0, st, v, a);
  } else if (trace) {
    if (m->fmt == 0) hipLaunchKernelGGL((render_k<0, true>), grd, dim3(64), 0, st, v, a);
    else if (m->fmt == 1) hipLaunchKernelGGL((render_k<1, true>), grd, dim3(64), 0, st, v, a);
    else hipLaunchKernelGGL((render_k<2, true>), grd, dim3(64), 0, st, v, a);
  } else {
    if (m->fmt == 0) hipLaunchKernelGGL((render_k<0, false>), grd, dim3(64), 0, st, v, a);
    else if (m->fmt == 1) hipLaunchKernelGGL((render_k<1, false>), grd, dim3(64), 0, st, v, a);
    else hipLaunchKernelGGL((render_k<2, false>), grd, dim3(64), 0, st, v, a);
  }
  DTSDF_HIP(hipGetLastError());
  return DTSDF_OK;
}

extern "C" dtsdf_status dtsdf_render_batch(const dtsdf_map* m, int32_t n,
                                           const dtsdf_render_req* reqs, void* stream) {
  if (!m || n < 0 || (n > 0 && !reqs) || n > 4096) return DTSDF_E_INVAL;
  if (n == 0) return DTSDF_OK;
  hipStream_t st = (hipStream_t)stream;
  // descriptor block: counter (16 B) | prefix[n + 1] | RenderArgs[n]
  const size_t off_prefix = 16;
  const size_t off_args = (off_prefix + sizeof(int32_t) * (n + 1) + 63) & ~(size_t)63;
  const size_t bytes = off_args + sizeof(RenderArgs) * n;
  static_assert((16 + 4 * 4097 + 63 + sizeof(RenderArgs) * 4096) <= kStageHostBytes,
                "the largest batch fits one staging slot");
  RenderArgs args1;
  int64_t total = 0;
  bool trace = false;
  for (int r = 0; r < n; ++r) {
    if (!fill_args(&reqs[r].intr, reqs[r].T_world_cam, reqs[r].z_near, reqs[r].z_far,
                   &reqs[r].out, args1))
      return DTSDF_E_INVAL;
    trace = trace || args1.trace_bricks || args1.trace_color || args1.trace_slots ||
            args1.trace_counts;
    total += args1.tiles;
    if (total > (int64_t)1 << 30) return DTSDF_E_INVAL;
  }
  Stage* sg = nullptr;
  dtsdf_status rs = stage_acquire(&sg);
  if (rs != DTSDF_OK) return rs;
  uint8_t* host = sg->host;
  std::memset(host, 0, off_args);
  int32_t* prefix = reinterpret_cast<int32_t*>(host + off_prefix);
  RenderArgs* args = reinterpret_cast<RenderArgs*>(host + off_args);
  total = 0;
  for (int r = 0; r < n; ++r) {
    fill_args(&reqs[r].intr, reqs[r].T_world_cam, reqs[r].z_near, reqs[r].z_far, &reqs[r].out,
              args[r]);
    prefix[r] = (int32_t)total;
    total += args[r].tiles;
  }
  prefix[n] = (int32_t)total;
  if (total <= kIlvBatchTiles) {
    // small batch: interleaved work tiles (see kIlvX)
    total = 0;
    for (int r = 0; r < n; ++r) {
      args[r].ilv = 1;
      prefix[r] = (int32_t)total;
      total += args[r].itiles;
    }
    prefix[n] = (int32_t)total;
  }
  uint8_t* dev = sg->dev;
  if (hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    rs = DTSDF_E_HIP;
  } else {
    // persistent waves: three per SIMD (the kernel's occupancy), four SIMDs per CU
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) !=
            hipSuccess || cus <= 0)
      cus = 170;
    const int wgs = (int)std::min<int64_t>(total, (int64_t)cus * 4 * 3);
    const MapView v = make_view(m);
    const RenderArgs* da = reinterpret_cast<const RenderArgs*>(dev + off_args);
    const int32_t* dp = reinterpret_cast<const int32_t*>(dev + off_prefix);
    int32_t* ctr = reinterpret_cast<int32_t*>(dev);
    if (m->regular) {
      if (trace)
        hipLaunchKernelGGL((render_batch_k<kRegularVolume, true>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
      else
        hipLaunchKernelGGL((render_batch_k<kRegularVolume, false>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
    } else if (trace) {
      if (m->fmt == 0)
        hipLaunchKernelGGL((render_batch_k<0, true>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
      else if (m->fmt == 1)
        hipLaunchKernelGGL((render_batch_k<1, true>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
      else
        hipLaunchKernelGGL((render_batch_k<2, true>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
    } else {
      if (m->fmt == 0)
        hipLaunchKernelGGL((render_batch_k<0, false>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
      else if (m->fmt == 1)
        hipLaunchKernelGGL((render_batch_k<1, false>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
      else
        hipLaunchKernelGGL((render_batch_k<2, false>), dim3(wgs), dim3(64), 0, st, v, da, dp, n, (int)total, ctr);
    }
    if (hipGetLastError() != hipSuccess) rs = DTSDF_E_HIP;
  }
  const dtsdf_status rr = stage_release(sg, st);
  return rs != DTSDF_OK ? rs : rr;
}
