// Driver of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer (test only):
// builds the oracle source into one executable and runs its integrate, requests, render
// (with the grazing classification), eval, export/import, recycle and combine entry points
// once on a small analytic scene (a sphere in front of a wall).  Exit status 0 and a
// silent sanitizer are the test.
#include "../oracle/dtsdf_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

// Camera-to-world pose on a circle of radius 1 m around the origin in the z = 0.1 plane,
// looking at the origin (OpenCV axes: x right, y down, z forward).
void circle_pose(double phi, double T[16]) {
  const double c[3] = {std::cos(phi), std::sin(phi), 0.1};
  double z[3] = {-c[0], -c[1], -c[2]};
  double nz = std::sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
  for (double& v : z) v /= nz;
  const double up[3] = {0, 0, 1};
  double x[3] = {z[1] * up[2] - z[2] * up[1], z[2] * up[0] - z[0] * up[2],
                 z[0] * up[1] - z[1] * up[0]};
  double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  for (double& v : x) v /= nx;
  const double y[3] = {z[1] * x[2] - z[2] * x[1], z[2] * x[0] - z[0] * x[2],
                       z[0] * x[1] - z[1] * x[0]};
  for (int r = 0; r < 3; ++r) {
    T[4 * r + 0] = x[r];
    T[4 * r + 1] = y[r];
    T[4 * r + 2] = z[r];
    T[4 * r + 3] = c[r];
  }
  T[12] = T[13] = T[14] = 0;
  T[15] = 1;
}

// Depth (along the optical axis) of a sphere of radius 0.2 m at the origin, in front of a
// plane 0.35 m behind the origin (as seen from the camera), for every pixel.
void analytic_depth(const double T[16], int W, int H, double f, double cx, double cy,
                    std::vector<float>& depth, std::vector<uint8_t>& rgb) {
  const double o[3] = {T[3], T[7], T[11]};
  const double back[3] = {-o[0], -o[1], 0.0};   // unit-ish direction away from the camera
  const double nb = std::sqrt(back[0] * back[0] + back[1] * back[1]);
  depth.assign((size_t)W * H, 0.f);
  rgb.assign((size_t)W * H * 3, 0);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      const double dc[3] = {(u - cx) / f, (v - cy) / f, 1.0};
      double d[3];
      for (int k = 0; k < 3; ++k) d[k] = T[4 * k] * dc[0] + T[4 * k + 1] * dc[1] + T[4 * k + 2] * dc[2];
      // sphere: |o + t d|^2 = r^2
      const double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double b = 2 * (o[0] * d[0] + o[1] * d[1] + o[2] * d[2]);
      const double c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - 0.04;
      const double disc = b * b - 4 * a * c;
      double t = 1e30;
      uint8_t col = 200;
      if (disc >= 0) t = (-b - std::sqrt(disc)) / (2 * a);
      // wall: <x, back/|back|> = 0.35
      const double dn = (d[0] * back[0] + d[1] * back[1]) / nb;
      if (dn > 1e-9) {
        const double tw = (0.35 - (o[0] * back[0] + o[1] * back[1]) / nb) / dn;
        if (tw > 0 && tw < t) {
          t = tw;
          col = 90;
        }
      }
      if (t < 1e29) {
        depth[(size_t)v * W + u] = (float)t;   // dc has z = 1: t is the depth
        for (int ch = 0; ch < 3; ++ch) rgb[3 * ((size_t)v * W + u) + ch] = (uint8_t)(col + 20 * ch);
      }
    }
}

}  // namespace

int main() {
  Params p{};
  p.voxel = 0.01;
  p.tau = 0.04;
  p.theta = kPi / 3;
  p.w_carve = 0.1;
  p.w_max = 63.75;
  p.w_min = 1e-4;
  p.step = 0.005;
  p.with_color = 1;
  void* h = orc_create(&p);
  const int W = 64, H = 48;
  const double f = 60.0, cx = 31.5, cy = 23.5;
  std::vector<float> depth;
  std::vector<uint8_t> rgb;
  const double phis[3] = {0.0, 0.4, -0.3};
  for (double phi : phis) {
    double T[16];
    circle_pose(phi, T);
    analytic_depth(T, W, H, f, cx, cy, depth, rgb);
    OrcStats st{};
    orc_integrate(h, depth.data(), rgb.data(), W, H, f, f, cx, cy, T, 1.0, &st, nullptr);
    std::printf("integrate phi=%.2f: %lld new bricks, %lld updates\n", phi,
                (long long)st.new_bricks, (long long)st.updated);
  }
  // block requests of one more frame, without fusing it
  double T[16];
  circle_pose(0.2, T);
  analytic_depth(T, W, H, f, cx, cy, depth, rgb);
  const int64_t cap = (int64_t)W * H * 6 * 64;
  std::vector<int32_t> keys(4 * cap);
  std::vector<uint8_t> border(cap), alloc(cap);
  const int64_t nreq = orc_requests(h, depth.data(), W, H, f, f, cx, cy, T, 1.0, keys.data(),
                                    border.data(), alloc.data(), cap, nullptr);
  // render every pixel with the grazing classification
  std::vector<int32_t> us, vs;
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      us.push_back(u);
      vs.push_back(v);
    }
  const int64_t n = (int64_t)us.size();
  std::vector<double> dep(n), vert(3 * n), nrm(3 * n), thit(n);
  std::vector<uint8_t> rgba(4 * n), mask(n), flags(n), touched((size_t)orc_num_bricks(h));
  std::vector<int64_t> khit(n);
  OrcRenderCfg cfg{0.2, 3.0, 1e-5, 1e-6, 1e-5, 2e-6, 1, 0.25 * 3.141592653589793 / 180.0, 0.5};
  orc_render(h, n, us.data(), vs.data(), f, f, cx, cy, T, &cfg, dep.data(), vert.data(),
             nrm.data(), rgba.data(), mask.data(), flags.data(), khit.data(), thit.data(),
             touched.data());
  int64_t hits = 0;
  for (uint8_t mk : mask) hits += mk;
  // eval at a few points
  const double xs[6] = {0.19, 0.0, 0.0, 0.0, 0.21, 0.02};
  const double rs[6] = {-1, 0, 0, 0, -1, 0};
  double fv[2];
  uint8_t def[2], fb[2];
  orc_eval(h, 2, xs, rs, fv, def, fb);
  // export, import into a second map, recycle
  const int64_t nb = orc_num_bricks(h);
  std::vector<int32_t> ek(4 * nb);
  std::vector<float> es(512 * nb), ew(512 * nb), ewc(512 * nb);
  std::vector<uint8_t> ergb(3 * 512 * nb), eborder(512 * nb);
  orc_export(h, ek.data(), es.data(), ew.data(), ergb.data(), ewc.data(), eborder.data());
  void* h2 = orc_create(&p);
  orc_import(h2, nb, ek.data(), es.data(), ew.data(), ergb.data(), ewc.data());
  const int64_t freed = orc_recycle(h2, 0.9);
  // combined (single-direction) volume of the first map for this pose
  Params ps = p;
  ps.single_direction = 1;
  void* hv = orc_create(&ps);
  orc_combine(h, hv, T, T, W, H, f, f, cx, cy, 0.125, 0, 1e-5, 1e-6);
  orc_combine(h, hv, T, T, W, H, f, f, cx, cy, 0.125, 1, 1e-5, 1e-6);
  std::printf("requests %lld, hits %lld of %lld, eval %d/%d, bricks %lld, recycled %lld, "
              "volume bricks %lld\n",
              (long long)nreq, (long long)hits, (long long)n, (int)def[0], (int)def[1],
              (long long)nb, (long long)freed, (long long)orc_num_bricks(hv));
  orc_destroy(hv);
  orc_destroy(h2);
  orc_destroy(h);
  return hits > 0 && nb > 0 ? 0 : 3;
}
