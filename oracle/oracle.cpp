// CPU oracle of the stereo VIO frontend (VkVIO, arXiv 2609.30459, Sec. III).
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library; the product path never does.
// It is a plain, slow, loop-by-loop statement of what the frontend computes and
// shares no code, header or table with the GPU implementation.
//
// Precision: the pyramid and the detector are integer. The tracker is a template
// on its real type; the float instantiation takes the tracked/lost decisions in
// the same precision as the GPU kernels (the workloads fix FP32), the double
// instantiation serves the closed-form and brute-force pins.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <vector>

namespace orc {

// ----------------------------------------------------------------------------
// Images
// ----------------------------------------------------------------------------
struct Img {
  int w = 0, h = 0;
  std::vector<uint8_t> p;
  int at(int x, int y) const { return p[(size_t)y * w + x]; }
};

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ----------------------------------------------------------------------------
// Pyramid, Sec. III-C, eqs. (1)-(3).
// Horizontal pass V(x, y) = sum_i w_i L(2x+i, y), then vertical pass
// L'(x, y) = (sum_j w_j V(x, 2y+j) + 128) >> 8 with w = [1 4 6 4 1].
// Reading: eq. (1) rounds to nearest and eq. (3) shifts; the +128 bias before
// the shift satisfies both (round half up). Taps outside the image are clamped
// to the edge. The next level has floor(W/2) x floor(H/2) pixels.
// ----------------------------------------------------------------------------
static const int BINOM[5] = {1, 4, 6, 4, 1};

Img downsample(const Img& s) {
  Img d;
  d.w = s.w / 2;
  d.h = s.h / 2;
  d.p.assign((size_t)d.w * d.h, 0);
  // eq. (2): V has d.w columns and s.h rows
  std::vector<uint32_t> V((size_t)d.w * s.h);
  for (int y = 0; y < s.h; ++y)
    for (int x = 0; x < d.w; ++x) {
      uint32_t acc = 0;
      for (int i = -2; i <= 2; ++i) acc += BINOM[i + 2] * s.at(clampi(2 * x + i, 0, s.w - 1), y);
      V[(size_t)y * d.w + x] = acc;
    }
  // eq. (3)
  for (int y = 0; y < d.h; ++y)
    for (int x = 0; x < d.w; ++x) {
      uint32_t acc = 0;
      for (int j = -2; j <= 2; ++j) acc += BINOM[j + 2] * V[(size_t)clampi(2 * y + j, 0, s.h - 1) * d.w + x];
      d.p[(size_t)y * d.w + x] = (uint8_t)((acc + 128) >> 8);
    }
  return d;
}

std::vector<Img> pyramid(const Img& l0, int L) {
  std::vector<Img> pyr{l0};
  for (int l = 1; l < L; ++l) pyr.push_back(downsample(pyr.back()));
  return pyr;
}

// ----------------------------------------------------------------------------
// FAST-9 score, Sec. III-D. A pixel is a corner at threshold tau if at least 9
// contiguous pixels of the 16-pixel Bresenham circle of radius 3 are all
// brighter than I(p)+tau or all darker than I(p)-tau; the score is the largest
// such tau. With strict inequalities and integer tau this is
//   m = max over polarity and arc start of min over the 9 arc pixels of the
//       signed difference, score = max(m - 1, -1)  (-1: no tau >= 0 works).
// Circle order: start at (0,-3) and go clockwise (x right, y down).
// ----------------------------------------------------------------------------
static const int CIRCLE[16][2] = {{0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0},  {3, 1},  {2, 2},   {1, 3},
                                  {0, 3},  {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

int fast_score(const Img& I, int x, int y) {
  const int c = I.at(x, y);
  int d[16];
  for (int k = 0; k < 16; ++k) d[k] = I.at(x + CIRCLE[k][0], y + CIRCLE[k][1]) - c;
  int best = std::numeric_limits<int>::min();
  for (int pol = 0; pol < 2; ++pol)
    for (int s = 0; s < 16; ++s) {
      int m = std::numeric_limits<int>::max();
      for (int k = 0; k < 9; ++k) {
        const int v = pol == 0 ? d[(s + k) % 16] : -d[(s + k) % 16];
        m = std::min(m, v);
      }
      best = std::max(best, m);
    }
  return std::max(best - 1, -1);
}

// score map; pixels closer than 3 px to the border have no score (INT_MIN)
std::vector<int> score_map(const Img& I) {
  std::vector<int> S((size_t)I.w * I.h, std::numeric_limits<int>::min());
  for (int y = 3; y < I.h - 3; ++y)
    for (int x = 3; x < I.w - 3; ++x) S[(size_t)y * I.w + x] = fast_score(I, x, y);
  return S;
}

// ----------------------------------------------------------------------------
// Grid detection, Sec. III-D. Cells of C x C pixels from (0,0), row-major,
// partial cells included. Per cell the threshold sequence is walked in order;
// at each threshold the survivors of a strict 3x3 non-maximum suppression with
// score >= threshold are ranked by (score desc, y asc, x asc) and the first k
// kept; the walk stops once k are found. Candidates keep an edge margin E.
// ----------------------------------------------------------------------------
struct Corner {
  int x, y, score;
};

static bool nms_survivor(const std::vector<int>& S, int w, int x, int y) {
  const int s = S[(size_t)y * w + x];
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      if (!dx && !dy) continue;
      if (!(s > S[(size_t)(y + dy) * w + x + dx])) return false;
    }
  return true;
}

static bool corner_before(const Corner& a, const Corner& b) {
  if (a.score != b.score) return a.score > b.score;
  if (a.y != b.y) return a.y < b.y;
  return a.x < b.x;
}

// winners[cell] = up to k corners in rank order. mask (w*h bytes, or NULL):
// the caller's detection mask (the mask buffer of Fig. 2); a corner on a
// nonzero mask pixel is dropped after non-maximum suppression, so it still
// suppresses its neighbours but never becomes a winner.
std::vector<std::vector<Corner>> detect_cells(const Img& I, int C, int k, const int* thr, int nthr, int E,
                                              bool single_pass, const uint8_t* mask = nullptr) {
  const std::vector<int> S = score_map(I);
  const int ncx = (I.w + C - 1) / C, ncy = (I.h + C - 1) / C;
  std::vector<std::vector<Corner>> win((size_t)ncx * ncy);
  for (int cy = 0; cy < ncy; ++cy)
    for (int cx = 0; cx < ncx; ++cx) {
      const int x0 = std::max(cx * C, E), x1 = std::min(cx * C + C - 1, I.w - 1 - E);
      const int y0 = std::max(cy * C, E), y1 = std::min(cy * C + C - 1, I.h - 1 - E);
      std::vector<Corner> kept;
      for (int ti = single_pass ? nthr - 1 : 0; ti < nthr; ++ti) {
        std::vector<Corner> surv;
        for (int y = y0; y <= y1; ++y)
          for (int x = x0; x <= x1; ++x) {
            const int s = S[(size_t)y * I.w + x];
            if (s >= thr[ti] && nms_survivor(S, I.w, x, y) && !(mask && mask[(size_t)y * I.w + x]))
              surv.push_back({x, y, s});
          }
        std::sort(surv.begin(), surv.end(), corner_before);
        if ((int)surv.size() > k) surv.resize(k);
        kept = surv;
        if ((int)kept.size() >= k) break;
      }
      win[(size_t)cy * ncx + cx] = kept;
    }
  return win;
}

// ----------------------------------------------------------------------------
// Patch tracker, Sec. III-E, eqs. (4)-(5).
// Pattern: 52 half-integer offsets (u, v) in {+-0.5 .. +-3.5}^2 with
// u^2 + v^2 <= 16, ordered by v then u.
// ----------------------------------------------------------------------------
struct Pattern {
  float u[52], v[52];
  Pattern() {
    int n = 0;
    for (int j = 0; j < 8; ++j)
      for (int i = 0; i < 8; ++i) {
        const float uu = -3.5f + i, vv = -3.5f + j;
        if (uu * uu + vv * vv <= 16.0f) {
          u[n] = uu;
          v[n] = vv;
          ++n;
        }
      }
  }
};
static const Pattern PAT;

enum Status { TRACKED = 0, DETECTED = 1, MATCHED = 2, LOST_FB = 3, LOST_OOB = 4, LOST_DEGENERATE = 5, LOST_CAP = 6 };

template <class R>
static bool in_domain(const Img& I, R x, R y) {
  return x >= R(0) && x <= R(I.w - 1) && y >= R(0) && y <= R(I.h - 1);
}

// bilinear interpolation, defined on [0, W-1] x [0, H-1]
template <class R>
static R bilinear(const Img& I, R x, R y) {
  const int ix = std::min((int)std::floor(x), I.w - 2), iy = std::min((int)std::floor(y), I.h - 2);
  const R fx = x - R(ix), fy = y - R(iy);
  const R a = R(I.at(ix, iy)), b = R(I.at(ix + 1, iy)), c = R(I.at(ix, iy + 1)), d = R(I.at(ix + 1, iy + 1));
  return (R(1) - fy) * ((R(1) - fx) * a + fx * b) + fy * ((R(1) - fx) * c + fx * d);
}

template <class R>
struct Template {
  bool fits = false, valid = false;
  R T[52], G[52][3];
  R H[3][3], Hinv[3][3];
};

// 3x3 inverse by cofactors; returns the determinant
template <class R>
static R inverse3(const R m[3][3], R inv[3][3]) {
  const R c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
  const R c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
  const R c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
  const R det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
  const R id = R(1) / det;
  inv[0][0] = c00 * id;
  inv[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
  inv[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
  inv[1][0] = c01 * id;
  inv[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
  inv[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
  inv[2][0] = c02 * id;
  inv[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
  inv[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
  return det;
}

// Template on image I at (px, py): samples I_i = I(p + x_i), gradient by central
// differences of bilinear samples at +-1 px, mean-normalised (Sec. III-E):
// T_i = I_i / mean, g_i = grad I_i / mean, J_i = [gx, gy, gy u_i - gx v_i],
// H = sum J_i^T J_i, G_i = H^-1 J_i^T. Invalid if the mean is not positive,
// H is near singular (det <= 1e-6 (tr/3)^3) or a gain is not finite.
template <class R>
static Template<R> make_template(const Img& I, R px, R py) {
  Template<R> t;
  R Iv[52], gx[52], gy[52];
  for (int i = 0; i < 52; ++i) {
    const R sx = px + R(PAT.u[i]), sy = py + R(PAT.v[i]);
    if (!in_domain(I, sx - R(1), sy) || !in_domain(I, sx + R(1), sy) || !in_domain(I, sx, sy - R(1)) ||
        !in_domain(I, sx, sy + R(1)))
      return t;
  }
  t.fits = true;
  for (int i = 0; i < 52; ++i) {
    const R sx = px + R(PAT.u[i]), sy = py + R(PAT.v[i]);
    Iv[i] = bilinear(I, sx, sy);
    gx[i] = (bilinear(I, sx + R(1), sy) - bilinear(I, sx - R(1), sy)) / R(2);
    gy[i] = (bilinear(I, sx, sy + R(1)) - bilinear(I, sx, sy - R(1))) / R(2);
  }
  R sum = 0;
  for (int i = 0; i < 52; ++i) sum += Iv[i];
  const R mean = sum / R(52);
  if (!(mean > R(0))) return t;
  R J[52][3];
  for (int i = 0; i < 52; ++i) {
    t.T[i] = Iv[i] / mean;
    const R nx = gx[i] / mean, ny = gy[i] / mean;
    J[i][0] = nx;
    J[i][1] = ny;
    J[i][2] = ny * R(PAT.u[i]) - nx * R(PAT.v[i]);
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      R s = 0;
      for (int i = 0; i < 52; ++i) s += J[i][a] * J[i][b];
      t.H[a][b] = s;
    }
  const R det = inverse3(t.H, t.Hinv);
  const R tr3 = (t.H[0][0] + t.H[1][1] + t.H[2][2]) / R(3);
  if (!(det > R(1e-6) * tr3 * tr3 * tr3)) return t;
  for (int i = 0; i < 52; ++i)
    for (int a = 0; a < 3; ++a) {
      t.G[i][a] = t.Hinv[a][0] * J[i][0] + t.Hinv[a][1] * J[i][1] + t.Hinv[a][2] * J[i][2];
      if (!std::isfinite(t.G[i][a])) return t;
    }
  t.valid = true;
  return t;
}

// SE(2) exponential of (a, b, phi): rotation phi, translation V(phi) (a, b)
template <class R>
static void se2_exp(R a, R b, R phi, R& tx, R& ty) {
  R s, c;
  if (std::fabs(phi) < R(1e-4)) {
    s = R(1) - phi * phi / R(6);
    c = phi / R(2);
  } else {
    s = std::sin(phi) / phi;
    c = (R(1) - std::cos(phi)) / phi;
  }
  tx = s * a - c * b;
  ty = c * a + s * b;
}

template <class R>
struct Pose {
  R tx, ty, th;
};

template <class R>
struct PassOut {
  int status = TRACKED;
  Pose<R> T{};
  R resid = 0;
  R last_step = 0;
};

// One coarse-to-fine pass (Sec. III-E): template on `src` at p, warp
// initialised at `init` (level-0 position and rotation), exactly N Gauss-Newton
// iterations per level from level L-1 to 0 with t doubled between levels. A
// level whose template does not fit the image is skipped (level 0: LOST_OOB).
// Iteration (eqs. 4-5): x'_i = R(th) x_i + t; e_i = I'(x'_i)/mean' - T_i;
// delta = -sum_i G_i e_i; T <- T o exp(delta).
template <class R>
static PassOut<R> klt_pass(const std::vector<Img>& src, const std::vector<Img>& dst, R px, R py, Pose<R> init,
                           int L, int N) {
  PassOut<R> o;
  R tx = std::ldexp(init.tx, -(L - 1)), ty = std::ldexp(init.ty, -(L - 1)), th = init.th;
  for (int l = L - 1; l >= 0; --l) {
    if (l < L - 1) {
      tx = tx * R(2);
      ty = ty * R(2);
    }
    const Template<R> tm = make_template(src[l], std::ldexp(px, -l), std::ldexp(py, -l));
    if (!tm.fits) {
      if (l == 0) {
        o.status = LOST_OOB;
        return o;
      }
      continue;
    }
    if (!tm.valid) {
      o.status = LOST_DEGENERATE;
      return o;
    }
    const Img& I = dst[l];
    for (int it = 0; it < N; ++it) {
      const R c = std::cos(th), s = std::sin(th);
      R Iw[52];
      for (int i = 0; i < 52; ++i) {
        const R wx = (c * R(PAT.u[i]) - s * R(PAT.v[i])) + tx;
        const R wy = (s * R(PAT.u[i]) + c * R(PAT.v[i])) + ty;
        if (!in_domain(I, wx, wy)) {
          o.status = LOST_OOB;
          return o;
        }
        Iw[i] = bilinear(I, wx, wy);
      }
      R sum = 0;
      for (int i = 0; i < 52; ++i) sum += Iw[i];
      const R mean = sum / R(52);
      if (!(mean > R(0))) {
        o.status = LOST_OOB;
        return o;
      }
      R d0 = 0, d1 = 0, d2 = 0, ss = 0;
      for (int i = 0; i < 52; ++i) {
        const R e = Iw[i] / mean - tm.T[i];
        d0 -= tm.G[i][0] * e;
        d1 -= tm.G[i][1] * e;
        d2 -= tm.G[i][2] * e;
        ss += e * e;
      }
      if (l == 0 && it == N - 1) o.resid = std::sqrt(ss / R(52));
      R vx, vy;
      se2_exp(d0, d1, d2, vx, vy);
      tx = tx + (c * vx - s * vy);
      ty = ty + (s * vx + c * vy);
      th = th + d2;
      o.last_step = std::sqrt(d0 * d0 + d1 * d1);
    }
  }
  o.T = {tx, ty, th};
  return o;
}

template <class R>
struct TrackOut {
  int status;
  R x, y, th, fb, resid;
};

// Forward-backward tracking (Sec. III-E, Fig. 4). The backward pass rebuilds
// the template on the target at the forward result and starts from the inverse
// of the forward motion (position p, rotation -theta); the track is lost when
// the returned position is farther than fb_thr from p.
template <class R>
static TrackOut<R> track(const std::vector<Img>& src, const std::vector<Img>& dst, R px, R py, R ix, R iy, int L,
                         int N, R fb_thr, R ith = R(0)) {
  TrackOut<R> r{TRACKED, ix, iy, 0, 0, 0};
  const PassOut<R> f = klt_pass<R>(src, dst, px, py, {ix, iy, ith}, L, N);
  if (f.status != TRACKED) {
    r.status = f.status;
    return r;
  }
  r.x = f.T.tx;
  r.y = f.T.ty;
  r.th = f.T.th;
  r.resid = f.resid;
  const PassOut<R> b = klt_pass<R>(dst, src, f.T.tx, f.T.ty, {px, py, -f.T.th}, L, N);
  if (b.status != TRACKED) {
    r.status = b.status;
    return r;
  }
  const R dx = b.T.tx - px, dy = b.T.ty - py;
  r.fb = std::sqrt(dx * dx + dy * dy);
  r.status = r.fb > fb_thr ? LOST_FB : TRACKED;
  return r;
}

// ----------------------------------------------------------------------------
// Frontend pipeline per frame (Sec. III-B): pyramid, temporal tracking of every
// camera's live keypoints, detection on the first camera of each mono camera or
// stereo pair with cells masked by surviving tracks, stereo matching of the new
// detections into the second camera of the pair.
// ----------------------------------------------------------------------------
struct Params {
  uint32_t struct_size;
  int32_t levels, gn_iters, cell_size, k_per_cell, n_thresholds;
  int32_t thresholds[4];
  int32_t edge_margin, max_keypoints;
  float fb_threshold, disparity0;
  int32_t init_mode;  // 0 constant velocity, 1 learned
  int32_t learned_levels, learned_iters;
  float learned_rho;
  // predicted tracks (caller prediction or camera-model start): 0 levels = the
  // full budget; else this budget first, the full one from the same start when
  // the track is not kept or its residual RMS exceeds pred_rho
  int32_t pred_levels, pred_iters;
  float pred_rho;
  // cameras of a stereo frontend with 4k cameras: 0 = pairs (0,1), (2,3); 1 =
  // a star (0 -> 1, 2, 3): detection in the first camera of each group of
  // four, its new keypoints matched into the other three
  int32_t topology;
  // learned initialisation: budget of the fallback from the constant-velocity
  // start (0 levels = the full budget levels x gn_iters)
  int32_t learned_fb_levels, learned_fb_iters;
  // stereo start of a new keypoint's match: 0 = the disparity prior; 1 = the
  // neighbour start (the previous frame's nearest keypoint of the detecting
  // camera that also lives in the target camera lends its offset between the
  // two cameras), refined with stereo_levels x stereo_iters; without such a
  // keypoint the disparity prior and the full budget
  int32_t stereo_init, stereo_levels, stereo_iters;
};

struct Record {  // 40 bytes
  int64_t id;
  float x, y, theta, fb_err, resid_rms;
  int32_t age;
  int16_t camera, status;
  int32_t score;
};
static_assert(sizeof(Record) == 40, "record layout");

struct Keypoint {
  int64_t id;
  float x, y, px, py;
  int32_t age;
};

// ----------------------------------------------------------------------------
// Learned initialisation (a project addition; the paper initialises from the
// backend's prediction). An MLP maps 32 features of a keypoint to a
// displacement guess and a confidence:
//   features: the previous flows (x - px, y - py) / 16 of the 8 live tracks of
//             the camera nearest to the keypoint that have a flow (age >= 1),
//             by (squared distance, id) -- the keypoint's own track, at
//             distance 0, is the nearest when it has a flow -- zero when fewer
//             exist (16 values); and
//             the 16x16-pixel patch of the previous frame's level 0 around
//             round(p), mean-pooled over 4x4 cells: cell_mean / patch_mean - 1
//             (16 values), pixels clamped to the image.
//   network:  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
//             W1 128x32, W2 128x128, W3 3x128; guess (16 y0, 16 y1) px,
//             confidence sigmoid(y2).
//   precision: inputs, weights and the post-ReLU activations are rounded to
//             bfloat16 (round to nearest even); sums in float; biases float.
// ----------------------------------------------------------------------------
constexpr int MI = 32, MH = 128, MO = 3;
constexpr int OFF_W1 = 0, OFF_B1 = MH * MI, OFF_W2 = OFF_B1 + MH, OFF_B2 = OFF_W2 + MH * MH, OFF_W3 = OFF_B2 + MH,
              OFF_B3 = OFF_W3 + MO * MH, NPARAM = OFF_B3 + MO;
static_assert(NPARAM == 21123, "parameter count");

static float bf16r(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return x;  // inf / nan unchanged
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

// exact squared distance of two float positions (differences and squares are
// exact in double, so the ordering is the same on every platform)
static double dist2(float ax, float ay, float bx, float by) {
  const double dx = (double)ax - (double)bx, dy = (double)ay - (double)by;
  return dx * dx + dy * dy;
}

static void features_of(const std::vector<Keypoint>& live, const Img& prev0, float* out /* [n][32] */) {
  const int n = (int)live.size();
  for (int i = 0; i < n; ++i) {
    float* f = out + (size_t)i * MI;
    std::vector<std::pair<double, int64_t>> cand;
    std::vector<int> idx;
    for (int j = 0; j < n; ++j) {
      if (live[j].age < 1) continue;
      cand.push_back({dist2(live[j].x, live[j].y, live[i].x, live[i].y), live[j].id});
      idx.push_back(j);
    }
    std::vector<int> order(cand.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cand[a] < cand[b]; });
    for (int k = 0; k < 8; ++k) {
      if (k < (int)order.size()) {
        const Keypoint& q = live[idx[order[k]]];
        f[2 * k] = (q.x - q.px) * 0.0625f;
        f[2 * k + 1] = (q.y - q.py) * 0.0625f;
      } else {
        f[2 * k] = f[2 * k + 1] = 0.f;
      }
    }
    const int rx = (int)std::floor(live[i].x + 0.5f), ry = (int)std::floor(live[i].y + 0.5f);
    int64_t cell[16] = {0}, total = 0;
    for (int dy = 0; dy < 16; ++dy)
      for (int dx = 0; dx < 16; ++dx) {
        const int v = prev0.at(clampi(rx - 8 + dx, 0, prev0.w - 1), clampi(ry - 8 + dy, 0, prev0.h - 1));
        cell[(dy / 4) * 4 + dx / 4] += v;
        total += v;
      }
    for (int k = 0; k < 16; ++k)
      f[16 + k] = total > 0 ? (float)(cell[k] * 16) / (float)total - 1.f : 0.f;
  }
}

// Forward pass. bf16 = true: the GPU's rounding points; false: plain real R.
// Keeps the (rounded) activations for the backward pass.
template <class R>
static void mlp_forward(const float* P, const float* X, int n, bool bf16, R* Y, R* H1, R* H2) {
  auto wr = [&](float w) { return bf16 ? (R)bf16r(w) : (R)w; };
  for (int i = 0; i < n; ++i) {
    R x[MI], h1[MH], h2[MH];
    for (int k = 0; k < MI; ++k) x[k] = bf16 ? (R)bf16r(X[(size_t)i * MI + k]) : (R)X[(size_t)i * MI + k];
    for (int j = 0; j < MH; ++j) {
      R acc = 0;
      for (int k = 0; k < MI; ++k) acc += wr(P[OFF_W1 + j * MI + k]) * x[k];
      R h = acc + (R)P[OFF_B1 + j];
      h = h > 0 ? h : 0;
      h1[j] = bf16 ? (R)bf16r((float)h) : h;
    }
    for (int j = 0; j < MH; ++j) {
      R acc = 0;
      for (int k = 0; k < MH; ++k) acc += wr(P[OFF_W2 + j * MH + k]) * h1[k];
      R h = acc + (R)P[OFF_B2 + j];
      h = h > 0 ? h : 0;
      h2[j] = bf16 ? (R)bf16r((float)h) : h;
    }
    for (int c = 0; c < MO; ++c) {
      R acc = 0;
      for (int k = 0; k < MH; ++k) acc += wr(P[OFF_W3 + c * MH + k]) * h2[k];
      Y[(size_t)i * MO + c] = acc + (R)P[OFF_B3 + c];
    }
    if (H1) std::copy(h1, h1 + MH, H1 + (size_t)i * MH);
    if (H2) std::copy(h2, h2 + MH, H2 + (size_t)i * MH);
  }
}

// Loss over a batch (mean over samples): Huber (delta 1 px) on the guess
// (16 y0, 16 y1) against the target displacement, plus binary cross-entropy
// of the confidence logit y2 against c = [|guess - target| <= 2 px]. dY gets
// the gradient with respect to y.
template <class R>
static R mlp_loss(const R* Y, const float* tgt, int n, R* dY) {
  R loss = 0;
  for (int i = 0; i < n; ++i) {
    const R gx = (R)16 * Y[i * MO], gy = (R)16 * Y[i * MO + 1], z = Y[i * MO + 2];
    const R ex = gx - (R)tgt[2 * i], ey = gy - (R)tgt[2 * i + 1];
    const R hx = std::fabs(ex) <= 1 ? (R)0.5 * ex * ex : std::fabs(ex) - (R)0.5;
    const R hy = std::fabs(ey) <= 1 ? (R)0.5 * ey * ey : std::fabs(ey) - (R)0.5;
    const R c = std::sqrt(ex * ex + ey * ey) <= 2 ? (R)1 : (R)0;
    // softplus(z) - c z, written stably
    const R bce = (z > 0 ? z + std::log1p(std::exp(-z)) : std::log1p(std::exp(z))) - c * z;
    loss += hx + hy + bce;
    if (dY) {
      const R inv = (R)1 / (R)n;
      dY[i * MO] = (R)16 * std::max((R)-1, std::min((R)1, ex)) * inv;
      dY[i * MO + 1] = (R)16 * std::max((R)-1, std::min((R)1, ey)) * inv;
      dY[i * MO + 2] = ((R)1 / ((R)1 + std::exp(-z)) - c) * inv;
    }
  }
  return loss / (R)n;
}

// Backward pass from dY. bf16 = true: dY, dH2 and dH1 are rounded to bfloat16
// where the GPU rounds them (the operands of its matrix products); gradients
// of the biases sum the rounded values.
template <class R>
static void mlp_backward(const float* P, const float* X, const R* H1, const R* H2, const R* dYin, int n, bool bf16,
                         R* G /* NPARAM */) {
  auto rr = [&](R v) { return bf16 ? (R)bf16r((float)v) : v; };
  auto wr = [&](float w) { return bf16 ? (R)bf16r(w) : (R)w; };
  std::fill(G, G + NPARAM, (R)0);
  std::vector<R> dH2((size_t)n * MH), dH1((size_t)n * MH), dY((size_t)n * MO);
  for (size_t i = 0; i < dY.size(); ++i) dY[i] = rr(dYin[i]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < MH; ++j) {
      R acc = 0;
      for (int c = 0; c < MO; ++c) acc += dY[i * MO + c] * wr(P[OFF_W3 + c * MH + j]);
      dH2[(size_t)i * MH + j] = rr(H2[(size_t)i * MH + j] > 0 ? acc : (R)0);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < MH; ++j) {
      R acc = 0;
      for (int k = 0; k < MH; ++k) acc += dH2[(size_t)i * MH + k] * wr(P[OFF_W2 + k * MH + j]);
      dH1[(size_t)i * MH + j] = rr(H1[(size_t)i * MH + j] > 0 ? acc : (R)0);
    }
  for (int c = 0; c < MO; ++c) {
    for (int j = 0; j < MH; ++j) {
      R acc = 0;
      for (int i = 0; i < n; ++i) acc += dY[i * MO + c] * H2[(size_t)i * MH + j];
      G[OFF_W3 + c * MH + j] = acc;
    }
    R acc = 0;
    for (int i = 0; i < n; ++i) acc += dY[i * MO + c];
    G[OFF_B3 + c] = acc;
  }
  for (int j = 0; j < MH; ++j) {
    for (int k = 0; k < MH; ++k) {
      R acc = 0;
      for (int i = 0; i < n; ++i) acc += dH2[(size_t)i * MH + j] * H1[(size_t)i * MH + k];
      G[OFF_W2 + j * MH + k] = acc;
    }
    R acc = 0;
    for (int i = 0; i < n; ++i) acc += dH2[(size_t)i * MH + j];
    G[OFF_B2 + j] = acc;
  }
  for (int j = 0; j < MH; ++j) {
    for (int k = 0; k < MI; ++k) {
      R acc = 0;
      for (int i = 0; i < n; ++i) {
        const R x = bf16 ? (R)bf16r(X[(size_t)i * MI + k]) : (R)X[(size_t)i * MI + k];
        acc += dH1[(size_t)i * MH + j] * x;
      }
      G[OFF_W1 + j * MI + k] = acc;
    }
    R acc = 0;
    for (int i = 0; i < n; ++i) acc += dH1[(size_t)i * MH + j];
    G[OFF_B1 + j] = acc;
  }
}

// Adam (Kingma & Ba) on the float master parameters, step t >= 1.
static void adam(float* P, const float* G, float* m, float* v, int t, float lr, float b1, float b2, float eps) {
  const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
  for (int i = 0; i < NPARAM; ++i) {
    m[i] = b1 * m[i] + (1.f - b1) * G[i];
    v[i] = b2 * v[i] + (1.f - b2) * G[i] * G[i];
    const float mh = m[i] / c1, vh = v[i] / c2;
    P[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
}

// ----------------------------------------------------------------------------
// Camera-model initialisation, Sec. III-E: the forward warp starts from the
// pattern projected into the new image through the camera model, using the
// predicted pose and the keypoint's inverse depth.
//
// Pinhole camera with focal lengths (fx, fy) and principal point (cx, cy). The
// pixel p at inverse depth rho is the point X = ((px-cx)/fx, (py-cy)/fy, 1)/rho
// of the previous camera frame; the new camera frame holds X' = R X + t, seen
// at the pixel (fx X'x/X'z + cx, fy X'y/X'z + cy). A point must lie in front
// of the new camera: rho X'z > 1e-6 (else the keypoint keeps its usual start).
// The start of the SE(2) warp is the projection of p, with the rotation of the
// image x axis under the same mapping: the angle of proj(p + (1, 0)) - proj(p),
// both at the keypoint's inverse depth.
// ----------------------------------------------------------------------------
// A camera's projection model: pinhole (u = fx X/Z + cx, v = fy Y/Z + cy), or
// the equidistant fisheye model of Kannala and Brandt with four coefficients
// (KB4), which maps the angle theta between a ray and the optical axis to the
// radius theta_d = theta (1 + k1 theta^2 + k2 theta^4 + k3 theta^6 + k4
// theta^8) on the normalised image plane. Sec. III-E names only "the camera
// model"; pinhole and KB4 cover the calibrations of the paper's datasets.
struct CamModel {
  int kb4 = 0;
  double fx = 0, fy = 0, cx = 0, cy = 0;
  double k[4] = {};
};

struct Motion {
  bool on = false;
  CamModel src, dst;                // back-projecting and projecting camera (the same one for a temporal motion)
  double R[9] = {}, t[3] = {};
  double rho = 0;                   // inverse depth of keypoints without their own
  std::map<int64_t, double> depth;  // per-keypoint inverse depth, by id
};

// KB4 radius polynomial and its derivative at theta
static double kb4_radius(const CamModel& m, double th, double* deriv) {
  const double t2 = th * th;
  const double poly = 1 + t2 * (m.k[0] + t2 * (m.k[1] + t2 * (m.k[2] + t2 * m.k[3])));
  if (deriv) *deriv = 1 + t2 * (3 * m.k[0] + t2 * (5 * m.k[1] + t2 * (7 * m.k[2] + t2 * 9 * m.k[3])));
  return th * poly;
}

// The point at inverse depth rho on the ray of pixel (x, y): for the pinhole
// model at depth Z = 1 / rho, for KB4 at distance 1 / rho along the unit ray
// (a fisheye ray may leave the half-space Z > 0). KB4 inverts the radius
// polynomial by Newton's method from theta = theta_d; false when it does not
// converge to a root below pi where the radius rises with slope at least
// KB4_MIN_SLOPE (near the fold of the polynomial a pixel step turns the ray
// by 1 / slope times as much as on the axis: the ray is ill-conditioned and
// the keypoint keeps its usual start).
constexpr double KB4_MIN_SLOPE = 0.05;
static bool unproject(const CamModel& m, double rho, double x, double y, double X[3]) {
  const double a = (x - m.cx) / m.fx, b = (y - m.cy) / m.fy;
  if (!m.kb4) {
    X[0] = a / rho;
    X[1] = b / rho;
    X[2] = 1.0 / rho;
    return true;
  }
  const double td = std::sqrt(a * a + b * b);
  double th = td, d = 1;
  bool conv = false;
  for (int it = 0; it < 100 && !conv; ++it) {
    const double f = kb4_radius(m, th, &d) - td;
    if (!(d > 0)) return false;
    const double step = f / d;
    th -= step;
    conv = std::fabs(step) <= 1e-15 * (1 + th);
  }
  kb4_radius(m, th, &d);
  if (!conv || !(th >= 0) || !(th < M_PI) || !(d >= KB4_MIN_SLOPE)) return false;
  const double s = td > 0 ? std::sin(th) / td : 1.0;  // sin(theta) / theta_d -> 1 on the axis
  X[0] = s * a / rho;
  X[1] = s * b / rho;
  X[2] = std::cos(th) / rho;
  return true;
}

// Pixel of camera-frame point X; false for a pinhole point not in front of
// the camera (rho Z <= 1e-6, rho the inverse depth it was built at) and for a
// KB4 point on the optical axis behind the camera or at the centre.
static bool project(const CamModel& m, double rho, const double X[3], double& u, double& v) {
  if (!m.kb4) {
    if (!(rho * X[2] > 1e-6)) return false;
    u = m.fx * X[0] / X[2] + m.cx;
    v = m.fy * X[1] / X[2] + m.cy;
    return true;
  }
  const double r = std::sqrt(X[0] * X[0] + X[1] * X[1]);
  if (!(r > 0)) {
    if (!(X[2] > 0)) return false;
    u = m.cx;
    v = m.cy;
    return true;
  }
  const double rd = kb4_radius(m, std::atan2(r, X[2]), nullptr) / r;
  u = m.fx * rd * X[0] + m.cx;
  v = m.fy * rd * X[1] + m.cy;
  return true;
}

static bool project_pixel(const Motion& m, double rho, double x, double y, double& ox, double& oy) {
  double X[3], Xn[3];
  if (!unproject(m.src, rho, x, y, X)) return false;
  for (int i = 0; i < 3; ++i) Xn[i] = m.R[3 * i] * X[0] + m.R[3 * i + 1] * X[1] + m.R[3 * i + 2] * X[2] + m.t[i];
  return project(m.dst, rho, Xn, ox, oy);
}

static bool motion_start(const Motion& m, double rho, double x, double y, double& ix, double& iy, double& ith) {
  double x1, y1;
  if (!project_pixel(m, rho, x, y, ix, iy) || !project_pixel(m, rho, x + 1.0, y, x1, y1)) return false;
  ith = std::atan2(y1 - iy, x1 - ix);
  return true;
}

struct Camera {
  int w, h;
  std::vector<Img> prev;
  bool has_prev = false;
  std::vector<Keypoint> live;  // ascending id
};

struct Frontend {
  Params P;
  int n_cams;
  bool stereo;
  std::vector<Camera> cams;
  int64_t next_id = 0;
  std::vector<Record> records;
  std::vector<float> mlp;  // learned initialisation parameters (NPARAM)
  int last_fallback = 0;
  std::vector<Motion> motion;  // per camera, for the next frame only
  std::vector<std::vector<uint8_t>> mask;  // per camera detection mask (empty: none)
  std::vector<Motion> stereo_ext;          // per target camera: the stereo matches' camera-model start
};

static Record make_record(int64_t id, int cam, int status, float x, float y, float th, float fb, float res,
                          int age, int score) {
  Record r;
  r.id = id;
  r.camera = (int16_t)cam;
  r.status = (int16_t)status;
  r.x = x;
  r.y = y;
  r.theta = th;
  r.fb_err = fb;
  r.resid_rms = res;
  r.age = age;
  r.score = score;
  return r;
}

struct Pred {
  int64_t id;
  int cam;
  float x, y;
};

// A caller prediction (id, camera, position in the new frame) replaces the
// constant-velocity initialisation of that keypoint (Sec. III-E: the warp is
// initialised from the backend's prediction).
static void push_frame(Frontend& F, const uint8_t* const* imgs, const int32_t* strides,
                       const std::vector<Pred>& preds) {
  const Params& P = F.P;
  const int L = P.levels, N = P.gn_iters;
  std::vector<std::vector<Img>> cur(F.n_cams);
  for (int c = 0; c < F.n_cams; ++c) {
    Img l0;
    l0.w = F.cams[c].w;
    l0.h = F.cams[c].h;
    l0.p.resize((size_t)l0.w * l0.h);
    for (int y = 0; y < l0.h; ++y) std::memcpy(&l0.p[(size_t)y * l0.w], imgs[c] + (size_t)y * strides[c], l0.w);
    cur[c] = pyramid(l0, L);
  }
  F.records.clear();
  F.last_fallback = 0;
  std::vector<std::vector<Record>> rec(F.n_cams);
  // the keypoints every camera held after the previous frame (the neighbour
  // stereo start looks them up)
  std::vector<std::vector<Keypoint>> prev_live(F.n_cams);
  for (int c = 0; c < F.n_cams; ++c) prev_live[c] = F.cams[c].live;
  const int fbL = P.learned_fb_levels > 0 ? P.learned_fb_levels : L;
  const int fbN = P.learned_fb_levels > 0 ? P.learned_fb_iters : N;
  // temporal tracking with the constant-velocity initialisation; a camera with
  // no previous frame carries its keypoints over unchanged (nothing to track
  // against) and reports no temporal records
  for (int c = 0; c < F.n_cams; ++c) {
    Camera& cam = F.cams[c];
    if (!cam.has_prev) continue;
    std::vector<Keypoint> surv;
    // learned initialisation: one guess per keypoint from the previous frame
    const bool learned = P.init_mode == 1;
    std::vector<float> guess;
    if (learned && !cam.live.empty()) {
      std::vector<float> X(cam.live.size() * MI), Y(cam.live.size() * MO);
      features_of(cam.live, cam.prev[0], X.data());
      mlp_forward<float>(F.mlp.data(), X.data(), (int)cam.live.size(), true, Y.data(), (float*)nullptr,
                         (float*)nullptr);
      guess = Y;
    }
    {
      for (size_t ki = 0; ki < cam.live.size(); ++ki) {
        const Keypoint& k = cam.live[ki];
        float ix = k.x + (k.x - k.px), iy = k.y + (k.y - k.py), ith = 0.f;
        bool predicted = false;
        for (const Pred& q : preds)
          if (q.cam == c && q.id == k.id) {
            ix = q.x;
            iy = q.y;
            predicted = true;
          }
        const Motion& mo = F.motion[c];
        if (!predicted && mo.on) {
          const auto it = mo.depth.find(k.id);
          double mx, my, mth;
          if (motion_start(mo, it != mo.depth.end() ? it->second : mo.rho, k.x, k.y, mx, my, mth)) {
            ix = (float)mx;
            iy = (float)my;
            ith = (float)mth;
            predicted = true;
          }
        }
        TrackOut<float> r;
        bool done = false;
        if (learned && !predicted) {
          // the tracker refines the guess on a smaller budget; a track that is
          // not kept, or keeps a residual above rho, falls back to the
          // constant-velocity initialisation with the fallback budget
          const float gx = k.x + 16.f * guess[ki * MO], gy = k.y + 16.f * guess[ki * MO + 1];
          r = track<float>(cam.prev, cur[c], k.x, k.y, gx, gy, P.learned_levels, P.learned_iters, P.fb_threshold);
          done = r.status == TRACKED && r.resid <= P.learned_rho;
          if (!done) {
            F.last_fallback++;
            r = track<float>(cam.prev, cur[c], k.x, k.y, ix, iy, fbL, fbN, P.fb_threshold, ith);
            done = true;
          }
        }
        if (predicted && P.pred_levels > 0) {
          // a predicted start needs a smaller search range: the short budget
          // first, the full one (from the same start) when it does not hold
          r = track<float>(cam.prev, cur[c], k.x, k.y, ix, iy, P.pred_levels, P.pred_iters, P.fb_threshold, ith);
          done = r.status == TRACKED && r.resid <= P.pred_rho;
          if (!done) F.last_fallback++;
        }
        if (!done) r = track<float>(cam.prev, cur[c], k.x, k.y, ix, iy, L, N, P.fb_threshold, ith);
        if (r.status == TRACKED) {
          surv.push_back({k.id, r.x, r.y, k.x, k.y, k.age + 1});
          rec[c].push_back(make_record(k.id, c, TRACKED, r.x, r.y, r.th, r.fb, r.resid, k.age + 1, -1));
        } else {
          rec[c].push_back(make_record(k.id, c, r.status, r.x, r.y, r.th, r.fb, r.resid, k.age, -1));
        }
      }
    }
    cam.live = surv;
  }
  // detection, selection and stereo matching per mono camera, stereo pair or
  // star group (the first camera detects, the others receive its matches)
  const int group = !F.stereo ? 1 : (P.topology == 1 && F.n_cams % 4 == 0 ? 4 : 2);
  for (int g = 0; g < F.n_cams; g += group) {
    Camera& left = F.cams[g];
    const Img& I0 = cur[g][0];
    const int C = P.cell_size, k = P.k_per_cell;
    const auto win = detect_cells(I0, C, k, P.thresholds, P.n_thresholds, P.edge_margin, false,
                                  F.mask[g].empty() ? nullptr : F.mask[g].data());
    const int ncx = (I0.w + C - 1) / C, ncy = (I0.h + C - 1) / C;
    std::vector<int> occ((size_t)ncx * ncy, 0);
    for (const Keypoint& kp : left.live) {
      const int cx = (int)std::floor(kp.x / (float)C), cy = (int)std::floor(kp.y / (float)C);
      if (cx >= 0 && cx < ncx && cy >= 0 && cy < ncy) occ[(size_t)cy * ncx + cx]++;
    }
    struct Cand {
      int cell, rank;
      Corner c;
    };
    std::vector<Cand> cand;
    for (int cell = 0; cell < ncx * ncy; ++cell) {
      if (occ[cell] >= k) continue;
      for (int r = 0; r < (int)win[cell].size(); ++r) cand.push_back({cell, r, win[cell][r]});
    }
    // global cap: keep the best (score desc, cell asc, rank asc)
    std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
      if (a.c.score != b.c.score) return a.c.score > b.c.score;
      if (a.cell != b.cell) return a.cell < b.cell;
      return a.rank < b.rank;
    });
    const int room = std::max(0, P.max_keypoints - (int)left.live.size());
    if ((int)cand.size() > room) cand.resize(room);
    // identifiers in cell order
    std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
      if (a.cell != b.cell) return a.cell < b.cell;
      return a.rank < b.rank;
    });
    std::vector<Keypoint> fresh;
    for (const Cand& cd : cand) {
      const Keypoint kp{F.next_id++, (float)cd.c.x, (float)cd.c.y, (float)cd.c.x, (float)cd.c.y, 0};
      fresh.push_back(kp);
      left.live.push_back(kp);
      rec[g].push_back(make_record(kp.id, g, DETECTED, kp.x, kp.y, 0, 0, 0, 0, cd.c.score));
    }
    for (int tc = g + 1; tc < g + group; ++tc) {
      Camera& right = F.cams[tc];
      const Motion& ext = F.stereo_ext[tc];
      // neighbour start: the keypoints of the previous frame that live in both
      // the detecting and this camera, in id order, with their offset between
      // the two cameras
      struct Pair {
        float x, y, dx, dy;
        int64_t id;
      };
      std::vector<Pair> pairs;
      if (P.stereo_init == 1 && !ext.on) {
        const std::vector<Keypoint>& ls = prev_live[g];
        for (const Keypoint& q : prev_live[tc]) {
          const auto it = std::lower_bound(ls.begin(), ls.end(), q.id,
                                           [](const Keypoint& a, int64_t id) { return a.id < id; });
          if (it != ls.end() && it->id == q.id) pairs.push_back({it->x, it->y, q.x - it->x, q.y - it->y, q.id});
        }
      }
      for (const Keypoint& kp : fresh) {
        // the projection through the rig's extrinsics (Sec. III-E), else the
        // neighbour start, else the disparity prior
        float ix = kp.x - P.disparity0, iy = kp.y, ith = 0.f;
        int sL = L, sN = N;
        double mx, my, mth;
        if (ext.on && motion_start(ext, ext.rho, kp.x, kp.y, mx, my, mth)) {
          ix = (float)mx;
          iy = (float)my;
          ith = (float)mth;
        } else if (!pairs.empty()) {
          // nearest by (squared distance, id)
          size_t best = 0;
          double bd = dist2(pairs[0].x, pairs[0].y, kp.x, kp.y);
          for (size_t q = 1; q < pairs.size(); ++q) {
            const double d = dist2(pairs[q].x, pairs[q].y, kp.x, kp.y);
            if (d < bd || (d == bd && pairs[q].id < pairs[best].id)) {
              bd = d;
              best = q;
            }
          }
          ix = kp.x + pairs[best].dx;
          iy = kp.y + pairs[best].dy;
          sL = P.stereo_levels;
          sN = P.stereo_iters;
        }
        const TrackOut<float> r = track<float>(cur[g], cur[tc], kp.x, kp.y, ix, iy, sL, sN, P.fb_threshold, ith);
        int st = r.status == TRACKED ? MATCHED : r.status;
        if (st == MATCHED && (int)right.live.size() >= P.max_keypoints) st = LOST_CAP;
        if (st == MATCHED) right.live.push_back({kp.id, r.x, r.y, r.x, r.y, 0});
        rec[tc].push_back(make_record(kp.id, tc, st, r.x, r.y, r.th, r.fb, r.resid, 0, -1));
      }
    }
  }
  for (int c = 0; c < F.n_cams; ++c) {
    F.cams[c].prev = cur[c];
    F.cams[c].has_prev = true;
    F.records.insert(F.records.end(), rec[c].begin(), rec[c].end());
    F.motion[c] = Motion();
  }
}

}  // namespace orc

// ============================================================================
// C ABI for the test suite
// ============================================================================
using namespace orc;

extern "C" {

static Img make_img(const uint8_t* p, int w, int h) {
  Img I;
  I.w = w;
  I.h = h;
  I.p.assign(p, p + (size_t)w * h);
  return I;
}

// Levels 0..L-1 packed one after another (level l is floor(W/2^l) x floor(H/2^l)).
int orc_pyramid(const uint8_t* img, int w, int h, int L, uint8_t* out) {
  if (!img || !out || w < 2 || h < 2 || L < 1) return -1;
  const auto pyr = pyramid(make_img(img, w, h), L);
  size_t off = 0;
  for (const Img& I : pyr) {
    std::memcpy(out + off, I.p.data(), I.p.size());
    off += I.p.size();
  }
  return 0;
}

// FAST score of every pixel at least 3 px from the border; INT32_MIN elsewhere.
int orc_fast_scores(const uint8_t* img, int w, int h, int32_t* out) {
  if (!img || !out || w < 7 || h < 7) return -1;
  const auto S = score_map(make_img(img, w, h));
  std::memcpy(out, S.data(), S.size() * sizeof(int32_t));
  return 0;
}

// Per-cell winners: out[(cell * k + r) * 3 + {0,1,2}] = x, y, score (-1 = none).
int orc_detect(const uint8_t* img, int w, int h, int C, int k, const int32_t* thr, int nthr, int E,
               int single_pass, const uint8_t* mask, int32_t* out) {
  if (!img || !out || !thr || C < 1 || k < 1 || nthr < 1) return -1;
  const auto win = detect_cells(make_img(img, w, h), C, k, thr, nthr, E, single_pass != 0, mask);
  for (size_t cell = 0; cell < win.size(); ++cell)
    for (int r = 0; r < k; ++r) {
      int32_t* o = out + (cell * k + r) * 3;
      if (r < (int)win[cell].size()) {
        o[0] = win[cell][r].x;
        o[1] = win[cell][r].y;
        o[2] = win[cell][r].score;
      } else {
        o[0] = o[1] = o[2] = -1;
      }
    }
  return 0;
}

// Forward-backward tracking of n keypoints from the pyramid of `src` to that of
// `dst` (both level-0 images w x h). double_prec selects the FP64 instantiation.
// out_f[i*5 + {0..4}] = x, y, theta, fb, resid; out_status[i].
// ith: the forward pass's start rotation per keypoint (NULL: 0).
int orc_track(const uint8_t* src, const uint8_t* dst, int w, int h, int L, int N, double fb_thr, int n,
              const double* px, const double* py, const double* ix, const double* iy, const double* ith,
              int double_prec, double* out_f, int32_t* out_status) {
  if (!src || !dst || L < 1 || N < 0 || n < 0) return -1;
  const auto S = pyramid(make_img(src, w, h), L), D = pyramid(make_img(dst, w, h), L);
  for (int i = 0; i < n; ++i) {
    const double th0 = ith ? ith[i] : 0.0;
    if (double_prec) {
      const auto r = track<double>(S, D, px[i], py[i], ix[i], iy[i], L, N, fb_thr, th0);
      out_status[i] = r.status;
      const double v[5] = {r.x, r.y, r.th, r.fb, r.resid};
      std::memcpy(out_f + 5 * i, v, sizeof v);
    } else {
      const auto r = track<float>(S, D, (float)px[i], (float)py[i], (float)ix[i], (float)iy[i], L, N,
                                  (float)fb_thr, (float)th0);
      out_status[i] = r.status;
      const double v[5] = {r.x, r.y, r.th, r.fb, r.resid};
      std::memcpy(out_f + 5 * i, v, sizeof v);
    }
  }
  return 0;
}

// One coarse-to-fine forward pass only (no backward check), FP64.
// out[i*6 + {0..5}] = tx, ty, theta, resid, last_step, status
int orc_klt_pass(const uint8_t* src, const uint8_t* dst, int w, int h, int L, int N, int n, const double* px,
                 const double* py, const double* ix, const double* iy, const double* ith, double* out) {
  if (!src || !dst || L < 1 || N < 0) return -1;
  const auto S = pyramid(make_img(src, w, h), L), D = pyramid(make_img(dst, w, h), L);
  for (int i = 0; i < n; ++i) {
    const auto r = klt_pass<double>(S, D, px[i], py[i], {ix[i], iy[i], ith[i]}, L, N);
    const double v[6] = {r.T.tx, r.T.ty, r.T.th, r.resid, r.last_step, (double)r.status};
    std::memcpy(out + 6 * i, v, sizeof v);
  }
  return 0;
}

// Template quantities at one point of a single image (no pyramid), FP64:
// out[0..8] = H, out[9..17] = H^-1, out[18] = fits, out[19] = valid.
int orc_template(const uint8_t* img, int w, int h, double px, double py, double* out) {
  const Img I = make_img(img, w, h);
  const auto t = make_template<double>(I, px, py);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      out[3 * a + b] = t.H[a][b];
      out[9 + 3 * a + b] = t.Hinv[a][b];
    }
  out[18] = t.fits;
  out[19] = t.valid;
  return 0;
}

int orc_pattern(float* u, float* v) {
  for (int i = 0; i < 52; ++i) {
    u[i] = PAT.u[i];
    v[i] = PAT.v[i];
  }
  return 52;
}

// SE(2) exponential (a, b, phi) -> translation part; FP64.
void orc_se2_exp(double a, double b, double phi, double* tx, double* ty) { se2_exp<double>(a, b, phi, *tx, *ty); }

double orc_inverse3(const double* m, double* inv) {
  double M[3][3], I[3][3];
  for (int i = 0; i < 9; ++i) M[i / 3][i % 3] = m[i];
  const double det = inverse3<double>(M, I);
  for (int i = 0; i < 9; ++i) inv[i] = I[i / 3][i % 3];
  return det;
}

// ---- frontend --------------------------------------------------------------
void* orc_fe_create(int n_cams, const int32_t* widths, const int32_t* heights, int stereo, const Params* p) {
  if (!p || p->struct_size != sizeof(Params) || n_cams < 1 || (stereo && n_cams % 2)) return nullptr;
  if (p->pred_levels < 0 || p->pred_levels > p->levels || (p->pred_levels > 0 && p->pred_iters < 1)) return nullptr;
  if (p->topology != 0 && p->topology != 1) return nullptr;
  if (p->learned_fb_levels < 0 || p->learned_fb_levels > p->levels ||
      (p->learned_fb_levels > 0 && p->learned_fb_iters < 1))
    return nullptr;
  if (p->stereo_init != 0 && p->stereo_init != 1) return nullptr;
  if (p->stereo_init == 1 && (p->stereo_levels < 1 || p->stereo_levels > p->levels || p->stereo_iters < 1))
    return nullptr;
  auto* F = new Frontend();
  F->P = *p;
  F->n_cams = n_cams;
  F->stereo = stereo != 0;
  F->cams.resize(n_cams);
  F->motion.resize(n_cams);
  F->mask.resize(n_cams);
  F->stereo_ext.resize(n_cams);
  for (int c = 0; c < n_cams; ++c) {
    F->cams[c].w = widths[c];
    F->cams[c].h = heights[c];
  }
  return F;
}

void orc_fe_destroy(void* h) { delete static_cast<Frontend*>(h); }

int orc_fe_push(void* h, const uint8_t* const* imgs, const int32_t* strides) {
  if (!h || !imgs || !strides) return -1;
  if (static_cast<Frontend*>(h)->P.init_mode == 1 && static_cast<Frontend*>(h)->mlp.empty()) return -5;
  push_frame(*static_cast<Frontend*>(h), imgs, strides, {});
  return 0;
}

// As orc_fe_push with n predictions: pred_id[i], pred_cam[i], pred_xy[2i..2i+1].
int orc_fe_push_pred(void* h, const uint8_t* const* imgs, const int32_t* strides, int n, const int64_t* pred_id,
                     const int32_t* pred_cam, const float* pred_xy) {
  if (!h || !imgs || !strides || n < 0) return -1;
  if (static_cast<Frontend*>(h)->P.init_mode == 1 && static_cast<Frontend*>(h)->mlp.empty()) return -5;
  std::vector<Pred> v;
  for (int i = 0; i < n; ++i) v.push_back({pred_id[i], pred_cam[i], pred_xy[2 * i], pred_xy[2 * i + 1]});
  push_frame(*static_cast<Frontend*>(h), imgs, strides, v);
  return 0;
}

// Camera model and predicted motion of camera `cam` for the next frame only:
// K = (fx, fy, cx, cy), R row-major and t with X_new = R X_prev + t, rho the
// inverse depth of keypoints not among the n (ids[i], rhos[i]).
// A camera model from its C form: K[0..3] = fx, fy, cx, cy, K[4] = 0 for the
// pinhole model or 1 for KB4 with coefficients K[5..8].
static bool cam_model(const double* K, CamModel& m) {
  if (!K || !(K[0] > 0) || !(K[1] > 0) || !(K[4] == 0 || K[4] == 1)) return false;
  m.fx = K[0];
  m.fy = K[1];
  m.cx = K[2];
  m.cy = K[3];
  m.kb4 = K[4] == 1;
  for (int i = 0; i < 4; ++i) {
    m.k[i] = m.kb4 ? K[5 + i] : 0.0;
    if (!std::isfinite(m.k[i])) return false;
  }
  return true;
}

int orc_fe_set_motion(void* h, int cam, const double* K, const double* R, const double* t, double rho, int n,
                      const int64_t* ids, const double* rhos) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || cam < 0 || cam >= F->n_cams || !R || !t || n < 0 || !(rho > 0)) return -1;
  Motion m;
  if (!cam_model(K, m.src)) return -1;
  m.on = true;
  m.dst = m.src;
  for (int i = 0; i < 9; ++i) m.R[i] = R[i];
  for (int i = 0; i < 3; ++i) m.t[i] = t[i];
  m.rho = rho;
  for (int i = 0; i < n; ++i) {
    if (!(rhos[i] > 0)) return -1;
    m.depth[ids[i]] = rhos[i];
  }
  F->motion[cam] = m;
  return 0;
}

// The camera-model start of n keypoints: out[3i..3i+2] = x, y, theta and
// ok[i] = 1, or ok[i] = 0 when a projection is undefined (see project()).
// K, Kq: camera models (9 values each, as cam_model) of the back-projecting
// camera and of the camera projected into (NULL: K, the same camera).
int orc_motion_start(const double* K, const double* R, const double* t, int n, const double* x, const double* y,
                     const double* rho, double* out, int32_t* ok, const double* Kq) {
  if (!R || !t || n < 0) return -1;
  Motion m;
  if (!cam_model(K, m.src) || !cam_model(Kq ? Kq : K, m.dst)) return -1;
  for (int i = 0; i < 9; ++i) m.R[i] = R[i];
  for (int i = 0; i < 3; ++i) m.t[i] = t[i];
  for (int i = 0; i < n; ++i) {
    double ix = 0, iy = 0, ith = 0;
    ok[i] = motion_start(m, rho[i], x[i], y[i], ix, iy, ith) ? 1 : 0;
    out[3 * i] = ix;
    out[3 * i + 1] = iy;
    out[3 * i + 2] = ith;
  }
  return 0;
}

// Unprojection then projection through one camera model (9 values, as
// cam_model) of n pixels at inverse depth 1: out[2i..2i+1] = the pixel again,
// ok[i] = both steps defined; rays[3i..3i+2] (may be NULL) = the point.
int orc_camera_roundtrip(const double* K, int n, const double* x, const double* y, double* out, double* rays,
                         int32_t* ok) {
  CamModel m;
  if (!cam_model(K, m) || n < 0) return -1;
  for (int i = 0; i < n; ++i) {
    double X[3] = {0, 0, 0}, u = 0, v = 0;
    ok[i] = unproject(m, 1.0, x[i], y[i], X) && project(m, 1.0, X, u, v);
    out[2 * i] = u;
    out[2 * i + 1] = v;
    if (rays)
      for (int j = 0; j < 3; ++j) rays[3 * i + j] = X[j];
  }
  return 0;
}

// Projection of n camera-frame points through one camera model (9 values):
// out[2i..2i+1], ok[i] (the pinhole check at inverse depth 1).
int orc_camera_project(const double* K, int n, const double* X, double* out, int32_t* ok) {
  CamModel m;
  if (!cam_model(K, m) || n < 0) return -1;
  for (int i = 0; i < n; ++i) {
    double u = 0, v = 0;
    ok[i] = project(m, 1.0, X + 3 * i, u, v);
    out[2 * i] = u;
    out[2 * i + 1] = v;
  }
  return 0;
}

// Detection mask of camera `cam` (w*h bytes, row-major, nonzero = no
// detections there) for every following frame; NULL removes it.
int orc_fe_set_mask(void* h, int cam, const uint8_t* mask) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || cam < 0 || cam >= F->n_cams) return -1;
  const Camera& C = F->cams[cam];
  if (mask) F->mask[cam].assign(mask, mask + (size_t)C.w * C.h);
  else F->mask[cam].clear();
  return 0;
}

// Stereo extrinsics of target camera `cam` (a pair's right camera or a star's
// other camera), kept for every following frame: its matches of the detecting
// camera's new keypoints start at the projection of the keypoint at inverse
// depth rho, back-projected through Ks (the detecting camera), moved by
// X_target = R X + t and projected through Kt. R == NULL: the disparity prior.
int orc_fe_set_stereo(void* h, int cam, const double* Ks, const double* Kt, const double* R, const double* t,
                      double rho) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || cam < 0 || cam >= F->n_cams) return -1;
  if (!R) {
    F->stereo_ext[cam] = Motion();
    return 0;
  }
  Motion m;
  if (!t || !(rho > 0) || !cam_model(Ks, m.src) || !cam_model(Kt, m.dst)) return -1;
  m.on = true;
  for (int i = 0; i < 9; ++i) m.R[i] = R[i];
  for (int i = 0; i < 3; ++i) m.t[i] = t[i];
  m.rho = rho;
  F->stereo_ext[cam] = m;
  return 0;
}

int orc_fe_get(void* h, Record* out, int capacity, int* n_out) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || !n_out) return -1;
  *n_out = (int)F->records.size();
  if (capacity < (int)F->records.size()) return -4;
  std::memcpy(out, F->records.data(), F->records.size() * sizeof(Record));
  return 0;
}

// Replace camera `cam`'s live keypoints (id, x, y, px, py, age per entry, ids
// ascending) -- the keypoint state the host uploads before a frame.
int orc_fe_set_keypoints(void* h, int cam, int n, const int64_t* id, const float* xy_pxy, const int32_t* age) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || cam < 0 || cam >= F->n_cams || n < 0) return -1;
  std::vector<Keypoint> kps;
  for (int i = 0; i < n; ++i) {
    kps.push_back({id[i], xy_pxy[4 * i], xy_pxy[4 * i + 1], xy_pxy[4 * i + 2], xy_pxy[4 * i + 3], age[i]});
    F->next_id = std::max(F->next_id, id[i] + 1);
  }
  F->cams[cam].live = kps;
  return 0;
}

int orc_fe_get_keypoints(void* h, int cam, int capacity, int64_t* id, float* xy_pxy, int32_t* age) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || cam < 0 || cam >= F->n_cams) return -1;
  const auto& L = F->cams[cam].live;
  if ((int)L.size() > capacity) return -(int)L.size();
  for (size_t i = 0; i < L.size(); ++i) {
    id[i] = L[i].id;
    xy_pxy[4 * i] = L[i].x;
    xy_pxy[4 * i + 1] = L[i].y;
    xy_pxy[4 * i + 2] = L[i].px;
    xy_pxy[4 * i + 3] = L[i].py;
    age[i] = L[i].age;
  }
  return (int)L.size();
}

int64_t orc_fe_next_id(void* h) { return static_cast<Frontend*>(h)->next_id; }

int orc_fe_set_mlp(void* h, const float* params, int n) {
  auto* F = static_cast<Frontend*>(h);
  if (!F || !params || n != NPARAM) return -1;
  F->mlp.assign(params, params + n);
  return 0;
}

int orc_fe_last_fallback(void* h) { return static_cast<Frontend*>(h)->last_fallback; }

// ---- learned initialisation ------------------------------------------------
int orc_mlp_nparam() { return NPARAM; }

float orc_bf16(float x) { return bf16r(x); }

// Features of n live keypoints (id, x, y, px, py, age as in set_keypoints)
// over the previous frame's level-0 image prev (w x h).
int orc_features(int n, const int64_t* id, const float* xy_pxy, const int32_t* age, const uint8_t* prev, int w,
                 int h, float* out) {
  std::vector<Keypoint> live;
  for (int i = 0; i < n; ++i)
    live.push_back({id[i], xy_pxy[4 * i], xy_pxy[4 * i + 1], xy_pxy[4 * i + 2], xy_pxy[4 * i + 3], age[i]});
  features_of(live, make_img(prev, w, h), out);
  return 0;
}

// mode 0: float with bf16 rounding points; 1: double without rounding.
int orc_mlp_forward(const float* P, const float* X, int n, int mode, double* Y, double* H1, double* H2) {
  if (mode == 1) {
    mlp_forward<double>(P, X, n, false, Y, H1, H2);
    return 0;
  }
  std::vector<float> y((size_t)n * MO), h1((size_t)n * MH), h2((size_t)n * MH);
  mlp_forward<float>(P, X, n, true, y.data(), h1.data(), h2.data());
  std::copy(y.begin(), y.end(), Y);
  if (H1) std::copy(h1.begin(), h1.end(), H1);
  if (H2) std::copy(h2.begin(), h2.end(), H2);
  return 0;
}

// Loss and parameter gradient of a batch. mode as above.
double orc_mlp_loss_grad(const float* P, const float* X, const float* tgt, int n, int mode, double* G, double* dY_out) {
  if (mode == 1) {
    std::vector<double> y((size_t)n * MO), h1((size_t)n * MH), h2((size_t)n * MH), dy((size_t)n * MO);
    mlp_forward<double>(P, X, n, false, y.data(), h1.data(), h2.data());
    const double L = mlp_loss<double>(y.data(), tgt, n, dy.data());
    if (G) mlp_backward<double>(P, X, h1.data(), h2.data(), dy.data(), n, false, G);
    if (dY_out) std::copy(dy.begin(), dy.end(), dY_out);
    return L;
  }
  std::vector<float> y((size_t)n * MO), h1((size_t)n * MH), h2((size_t)n * MH), dy((size_t)n * MO), g(NPARAM);
  mlp_forward<float>(P, X, n, true, y.data(), h1.data(), h2.data());
  const float L = mlp_loss<float>(y.data(), tgt, n, dy.data());
  mlp_backward<float>(P, X, h1.data(), h2.data(), dy.data(), n, true, g.data());
  if (G) std::copy(g.begin(), g.end(), G);
  if (dY_out) std::copy(dy.begin(), dy.end(), dY_out);
  return L;
}

void orc_adam(float* P, const float* G, float* m, float* v, int t, float lr, float b1, float b2, float eps) {
  adam(P, G, m, v, t, lr, b1, b2, eps);
}

}  // extern "C"
