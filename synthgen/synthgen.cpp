// Seeded synthetic textured image sequences for the stereo frontend workloads.
//
// This module renders inputs only. It holds none of the frontend's arithmetic
// (no pyramid, no corner score, no patch alignment) and is shared by the CPU
// oracle and the GPU path purely as a data source. The paper evaluates on
// recorded datasets; these sequences stand in for them with the shapes, sizes
// and value distributions of the benchmark configurations.
//
// Random numbers: xoshiro256** seeded through SplitMix64 (Blackman & Vigna,
// public-domain generators, written here from their published definitions).
// Draw order per call: for every canvas in turn (background, blobs, rectangles,
// noise lattice), then one disparity plane per canvas, then the motion.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Rng {
  uint64_t s[4];
  static uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  explicit Rng(uint64_t seed) {
    uint64_t z = seed;
    for (auto& v : s) v = splitmix(z);
  }
  uint64_t next() {
    const uint64_t r = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
  }
  double uni() { return (double)(next() >> 11) * 0x1.0p-53; }          // [0,1)
  double uni(double a, double b) { return a + (b - a) * uni(); }        // [a,b)
  int integer(int lo, int hi) { return lo + (int)(uni() * (hi - lo + 1)); }  // [lo,hi]
  // uniform point in the disk of radius r (rejection from the square)
  void disk(double r, double& x, double& y) {
    for (;;) {
      x = uni(-1.0, 1.0);
      y = uni(-1.0, 1.0);
      if (x * x + y * y <= 1.0) break;
    }
    x *= r;
    y *= r;
  }
};

struct Canvas {
  int w = 0, h = 0;
  std::vector<float> v;
  float at(int x, int y) const { return v[(size_t)y * w + x]; }
  // bilinear sample with coordinates clamped to the canvas
  double sample(double x, double y) const {
    x = std::min(std::max(x, 0.0), (double)(w - 1));
    y = std::min(std::max(y, 0.0), (double)(h - 1));
    int ix = std::min((int)std::floor(x), w - 2), iy = std::min((int)std::floor(y), h - 2);
    double fx = x - ix, fy = y - iy;
    double a = at(ix, iy), b = at(ix + 1, iy), c = at(ix, iy + 1), d = at(ix + 1, iy + 1);
    return (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d);
  }
};

// Texture recipe: background U[20,235]; Gaussian blobs (sigma U[1.5,8], value
// U[20,235], alpha exp(-r^2/2sigma^2)); opaque axis-aligned rectangles (sides
// U[6,48], value U[20,235]) composited with exact pixel-area coverage; then a
// smooth value noise (integer lattice U{-4..4} every 8 px, bilinear).
void render_canvas(Rng& rng, Canvas& cv, int w, int h, double density) {
  cv.w = w;
  cv.h = h;
  const double bg = rng.uni(20.0, 235.0);
  cv.v.assign((size_t)w * h, (float)bg);
  const double area_units = (double)w * h / (320.0 * 240.0);
  const int n_blobs = (int)std::lround(64.0 * density * area_units);
  const int n_rects = (int)std::lround(32.0 * density * area_units);
  for (int b = 0; b < n_blobs; ++b) {
    const double cx = rng.uni(0.0, w), cy = rng.uni(0.0, h);
    const double sg = rng.uni(1.5, 8.0), val = rng.uni(20.0, 235.0);
    const double rad = 4.0 * sg, inv = 1.0 / (2.0 * sg * sg);
    const int x0 = std::max(0, (int)std::floor(cx - rad)), x1 = std::min(w - 1, (int)std::ceil(cx + rad));
    const int y0 = std::max(0, (int)std::floor(cy - rad)), y1 = std::min(h - 1, (int)std::ceil(cy + rad));
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) {
        const double r2 = (x - cx) * (x - cx) + (y - cy) * (y - cy);
        const double a = std::exp(-r2 * inv);
        float& p = cv.v[(size_t)y * w + x];
        p = (float)((1.0 - a) * p + a * val);
      }
  }
  for (int r = 0; r < n_rects; ++r) {
    const double rw = rng.uni(6.0, 48.0), rh = rng.uni(6.0, 48.0);
    const double rx = rng.uni(-rw, (double)w), ry = rng.uni(-rh, (double)h);
    const double val = rng.uni(20.0, 235.0);
    const int x0 = std::max(0, (int)std::floor(rx - 1)), x1 = std::min(w - 1, (int)std::ceil(rx + rw + 1));
    const int y0 = std::max(0, (int)std::floor(ry - 1)), y1 = std::min(h - 1, (int)std::ceil(ry + rh + 1));
    for (int y = y0; y <= y1; ++y) {
      const double oy = std::max(0.0, std::min(y + 0.5, ry + rh) - std::max(y - 0.5, ry));
      if (oy <= 0) continue;
      for (int x = x0; x <= x1; ++x) {
        const double ox = std::max(0.0, std::min(x + 0.5, rx + rw) - std::max(x - 0.5, rx));
        const double c = ox * oy;
        if (c <= 0) continue;
        float& p = cv.v[(size_t)y * w + x];
        p = (float)((1.0 - c) * p + c * val);
      }
    }
  }
  const int lw = w / 8 + 2, lh = h / 8 + 2;
  std::vector<int> lat((size_t)lw * lh);
  for (auto& q : lat) q = rng.integer(-4, 4);
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      const int gx = x / 8, gy = y / 8;
      const double fx = (x % 8) / 8.0, fy = (y % 8) / 8.0;
      const double n = (1 - fy) * ((1 - fx) * lat[(size_t)gy * lw + gx] + fx * lat[(size_t)gy * lw + gx + 1]) +
                       fy * ((1 - fx) * lat[(size_t)(gy + 1) * lw + gx] + fx * lat[(size_t)(gy + 1) * lw + gx + 1]);
      cv.v[(size_t)y * w + x] += (float)n;
    }
}

// Runs fn(y0, y1) over disjoint row bands on up to 16 threads; each pixel is
// a pure function of its position, so the image does not depend on the split.
template <class F>
void for_rows(int H, F fn) {
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int n = std::min(nt, std::max(1, H / 32));
  if (n == 1) {
    fn(0, H);
    return;
  }
  std::vector<std::thread> pool;
  for (int i = 0; i < n; ++i) pool.emplace_back(fn, H * i / n, H * (i + 1) / n);
  for (auto& t : pool) t.join();
}

inline uint8_t quantise(double v) {
  double r = std::floor(v + 0.5);
  return (uint8_t)std::min(255.0, std::max(0.0, r));
}

}  // namespace

extern "C" {

typedef struct {
  uint64_t seed;
  int32_t width, height;
  int32_t n_frames;
  int32_t n_canvases;   // one per mono camera or stereo pair
  int32_t stereo;       // extra views per canvas: 0 mono, 1 a stereo pair (left, right), 3 a star rig
                        // (a reference view and three views through their own disparity planes)
  int32_t warp_second;  // 1: two frames, the second is the bilinear warp of the first
  double density;       // 1.0 = 64 blobs + 32 rectangles per 320x240 area
  double max_t;         // per-frame translation bound (px)
  double max_rot_deg;   // per-frame rotation bound (deg), about the image centre
  double max_scale;     // per-frame relative scale bound
  double smooth;        // AR(1) coefficient of the per-frame motion increments
} sg_params;

// frames: [n_frames][n_cams][height][width] u8, n_cams = n_canvases * (1 + stereo)
// poses:  [n_frames][4] = (s, phi, ox, oy): canvas X = C + s R(phi) (x - c) + o
// planes: [n_canvases][max(1, stereo)][3] = (a, b, c): view v >= 1 of a canvas is
//         view(x, y) = reference(x + a x + b y + c, y) with plane v - 1
// warp:   [3] = (tx, ty, theta) of the second frame (warp_second mode only)
// Returns 0 on success, -1 on bad arguments.
int sg_render(const sg_params* p, uint8_t* frames, double* poses, double* planes, double* warp) {
  if (!p || !frames || !poses || !planes || !warp) return -1;
  const int W = p->width, H = p->height, T = p->n_frames;
  if (W < 16 || H < 16 || T < 1 || p->n_canvases < 1 || p->n_canvases > 8) return -1;
  if (p->stereo != 0 && p->stereo != 1 && p->stereo != 3) return -1;
  if (p->warp_second && (T != 2 || p->stereo)) return -1;
  Rng rng(p->seed);
  const int ncan = p->n_canvases;
  const int per = 1 + p->stereo;
  const int npl = p->stereo ? p->stereo : 1;  // planes per canvas
  const int ncam = ncan * per;
  const int CW = 3 * W, CH = 3 * H;
  std::vector<Canvas> canv(ncan);
  for (int k = 0; k < ncan; ++k) render_canvas(rng, canv[k], CW, CH, p->density);
  for (int k = 0; k < ncan * npl; ++k) {
    double a = 0, b = 0, c = 32.5;
    if (p->stereo) {
      for (;;) {
        a = rng.uni(-0.05, 0.05);
        b = rng.uni(-0.05, 0.05);
        c = rng.uni(5.0, 60.0);
        bool ok = true;
        const double xs[2] = {0.0, (double)(W - 1)}, ys[2] = {0.0, (double)(H - 1)};
        for (double x : xs)
          for (double y : ys) {
            const double d = a * x + b * y + c;
            if (d < 5.0 || d > 60.0) ok = false;
          }
        if (ok) break;
      }
    }
    planes[3 * k + 0] = a;
    planes[3 * k + 1] = b;
    planes[3 * k + 2] = c;
  }
  const double cx = (W - 1) * 0.5, cy = (H - 1) * 0.5;
  const double Cx = (CW - 1) * 0.5, Cy = (CH - 1) * 0.5;
  const double deg = M_PI / 180.0;
  // footprint bound: the image's rotated disk at scale <= 1.2 stays inside the canvas
  const double o_max = std::max(1.0, 0.5 * (1.5 * std::min(W, H) - 1.2 * 0.5 * std::hypot(W, H)));
  double s = 1.0, phi = 0.0, ox = 0.0, oy = 0.0;
  double vrot = 0.0, vs = 0.0, vtx = 0.0, vty = 0.0;
  warp[0] = warp[1] = warp[2] = 0.0;
  for (int t = 0; t < T; ++t) {
    if (t > 0 && !p->warp_second) {
      // smooth bounded increments, in image space: rotation about the centre,
      // relative scale and translation (convex combinations keep the bounds)
      const double a = p->smooth;
      double ux, uy;
      rng.disk(p->max_t, ux, uy);
      const double on = std::hypot(ox, oy);
      const double lam = std::min(1.0, on / o_max) * std::min(1.0, on / o_max);
      if (on > 0) {
        // pull back toward the canvas centre: o moves by -s' R(phi') u
        const double dx = ox / on, dy = oy / on;
        const double cr = std::cos(-phi), sr = std::sin(-phi);
        const double px = cr * dx - sr * dy, py = sr * dx + cr * dy;
        ux = (1 - lam) * ux + lam * p->max_t * px;
        uy = (1 - lam) * uy + lam * p->max_t * py;
      }
      const double ur = rng.uni(-p->max_rot_deg, p->max_rot_deg) * deg;
      double us = rng.uni(-p->max_scale, p->max_scale);
      const double ls = std::log(s);
      const double mu = std::min(1.0, std::fabs(ls) / std::log(1.15));
      us = (1 - mu * mu) * us + mu * mu * (ls > 0 ? p->max_scale : -p->max_scale);
      vtx = a * vtx + (1 - a) * ux;
      vty = a * vty + (1 - a) * uy;
      vrot = a * vrot + (1 - a) * ur;
      vs = a * vs + (1 - a) * us;
      // compose: x' = c + (1+vs) R(vrot) (x - c) + vt  (scene motion in the image)
      s = s / (1.0 + vs);
      phi = phi - vrot;
      const double cr = std::cos(phi), sr = std::sin(phi);
      ox -= s * (cr * vtx - sr * vty);
      oy -= s * (sr * vtx + cr * vty);
    }
    poses[4 * t + 0] = s;
    poses[4 * t + 1] = phi;
    poses[4 * t + 2] = ox;
    poses[4 * t + 3] = oy;
    const double cr = std::cos(phi), sr = std::sin(phi);
    for (int k = 0; k < ncan; ++k) {
      for (int side = 0; side < per; ++side) {
        uint8_t* img = frames + ((size_t)t * ncam + (size_t)k * per + side) * (size_t)W * H;
        if (p->warp_second && t == 1) continue;  // filled below
        const double* pl = planes + 3 * ((size_t)k * npl + (side ? side - 1 : 0));
        const double a = pl[0], b = pl[1], c = pl[2];
        const Canvas& cv = canv[k];
        for_rows(H, [&, img, side, a, b, c](int y0, int y1) {
          for (int y = y0; y < y1; ++y)
            for (int x = 0; x < W; ++x) {
              const double xl = side ? x + a * x + b * y + c : (double)x;
              const double dx = xl - cx, dy = y - cy;
              const double X = Cx + s * (cr * dx - sr * dy) + ox;
              const double Y = Cy + s * (sr * dx + cr * dy) + oy;
              img[(size_t)y * W + x] = quantise(cv.sample(X, Y));
            }
        });
      }
    }
  }
  if (p->warp_second) {
    double tx, ty;
    rng.disk(p->max_t, tx, ty);
    const double th = rng.uni(-p->max_rot_deg, p->max_rot_deg) * deg;
    warp[0] = tx;
    warp[1] = ty;
    warp[2] = th;
    const uint8_t* f0 = frames;
    uint8_t* f1 = frames + (size_t)W * H;
    const double cr = std::cos(th), sr = std::sin(th);
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        // inverse of x1 = c + R(th)(x0 - c) + t
        const double dx = x - cx - tx, dy = y - cy - ty;
        double sx = cx + cr * dx + sr * dy, sy = cy - sr * dx + cr * dy;
        sx = std::min(std::max(sx, 0.0), (double)(W - 1));
        sy = std::min(std::max(sy, 0.0), (double)(H - 1));
        const int ix = std::min((int)std::floor(sx), W - 2), iy = std::min((int)std::floor(sy), H - 2);
        const double fx = sx - ix, fy = sy - iy;
        const double v = (1 - fy) * ((1 - fx) * f0[(size_t)iy * W + ix] + fx * f0[(size_t)iy * W + ix + 1]) +
                         fy * ((1 - fx) * f0[(size_t)(iy + 1) * W + ix] + fx * f0[(size_t)(iy + 1) * W + ix + 1]);
        f1[(size_t)y * W + x] = quantise(v);
      }
  }
  return 0;
}

}  // extern "C"
