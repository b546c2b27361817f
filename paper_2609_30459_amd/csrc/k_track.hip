// Patch tracker for gfx950: inverse-compositional SE(2) alignment with a
// forward-backward check (Sec. III-E, eqs. 4-5, Fig. 4).
//
// One wave64 tracks one keypoint; lane i < 52 owns pattern point x_i (the 52
// half-integer offsets of the radius-4 disk, rows v = -3.5..3.5 of 4, 6, 8, 8,
// 8, 8, 6, 4 points), lanes 52..63 sit on an interior offset with weight 0 so
// every lane runs the same code. Every branch is taken on a wave vote, so a
// wave never diverges.
//
// A keypoint's time is its chain of dependent steps (2 passes x L levels x N
// iterations), each a gather, a reduction and a little wave-uniform math, with
// about one wave per SIMD at these sizes. The kernel is shaped for that chain:
//  * one copy of the alignment code per kernel: the learned attempt and the
//    plain one, and the forward and backward passes, run it in a loop with the
//    level count as an argument, so it is inlined and every descriptor field,
//    pyramid base pointer and warp parameter stays a scalar (SGPR) value;
//  * sums over the pattern are taken several at once: inside each 16-lane
//    row, four exchange stages (lane ^ 1, ^ 2 by quad permutes, rotations by 4
//    and 8) each halve the values a lane carries -- a lane keeps the half its
//    lane bit selects and adds its partner's copy of it -- until lane j of a
//    row holds sum j of that row; two row swaps (permlane32, permlane16) add
//    the four rows, and sum j is read from lane j. A fixed tree, so results
//    are deterministic, at about half the instructions of one reduction per
//    value;
//  * per iteration one fused reduction of (sum I'_i, sum G_i I'_i), since
//      delta = -sum_i G_i (I'_i / mean' - T_i) = c - (sum_i G_i I'_i) / mean'
//    with c = sum_i G_i T_i fixed per level;
//  * the templates of all levels of a pass are built together (they depend
//    only on the source image and the keypoint), so their loads and reductions
//    overlap; a point's five template samples (centre and the four neighbours
//    of the central difference) share one 4x4 pixel window, read as four
//    unaligned 32-bit rows;
//  * wave-uniform math uses the hardware reciprocal and sine/cosine, and a
//    series for the SE(2) exponential;
//  * gathers are global loads at a 32-bit offset from the level's scalar base,
//    through the L1 cache (the patch's lines stay hot across a level's
//    iterations).
// Decisions (template fit, degeneracy, leaving the image) are taken in the
// same order as a level-by-level pass, so the status is that of the paper's
// procedure.
//
// The same launch also runs the stereo matching of every detected cell winner
// (left camera -> right camera of the pair): those matches depend only on the
// current pyramids, so they run beside the temporal tracks instead of after the
// selection, and the selection kernel picks the ones it keeps.
#include <algorithm>

#include "fe_common.h"
#include "learn_ops.h"
#include "wave_ops.h"

// Multiply-adds are fused only within one expression (a * b + c), never
// across statements, so the rounding of every step follows from the source
// alone: the one- and two-keypoint-per-wave kernels, whose surrounding code
// differs, compute the same values.
#pragma clang fp contract(on)

namespace vio {
namespace {

constexpr int kW = 64;

typedef const __attribute__((address_space(1))) uint8_t* gbytes;
struct __attribute__((packed)) U16 {
  uint16_t v;
};
struct __attribute__((packed)) U32 {
  uint32_t v;
};

// unaligned 16- and 32-bit global loads at a 32-bit byte offset
__device__ __forceinline__ uint32_t ld16(gbytes p, uint32_t off) {
  return ((const __attribute__((address_space(1))) U16*)(p + off))->v;
}
__device__ __forceinline__ uint32_t ld32(gbytes p, uint32_t off) {
  return ((const __attribute__((address_space(1))) U32*)(p + off))->v;
}

__device__ __forceinline__ bool wave_all(bool p) { return __all(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __any(p); }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ void pattern_of(int lane, float& u, float& v, float& w) {
  // rows v = -3.5 .. 3.5 hold 4, 6, 8, 8, 8, 8, 6, 4 points; row starts 0, 4,
  // 10, 18, 26, 34, 42, 48 (52 in all)
  int r, base, n;
  if (lane < 4) r = 0, base = 0, n = 4;
  else if (lane < 10) r = 1, base = 4, n = 6;
  else if (lane < 42) r = 2 + (lane - 10) / 8, base = 10 + 8 * ((lane - 10) / 8), n = 8;
  else if (lane < 48) r = 6, base = 42, n = 6;
  else if (lane < 52) r = 7, base = 48, n = 4;
  else r = -1, base = 0, n = 0;
  if (r < 0) {
    u = 0.5f;
    v = 0.5f;
    w = 0.f;
    return;
  }
  v = -3.5f + (float)r;
  u = -0.5f * (float)(n - 1) + (float)(lane - base);
  w = 1.f;
}

struct Level {
  gbytes p;
  int pitch, w, h;
};

// x in [0, W-1] and y in [0, H-1], without short-circuit branches
__device__ __forceinline__ bool in_dom(const Level& I, float x, float y) {
  return (x >= 0.f) & (x <= (float)(I.w - 1)) & (y >= 0.f) & (y <= (float)(I.h - 1));
}

// bilinear interpolation on [0, W-1] x [0, H-1]: ix = min(floor(x), W-2),
// fx = x - ix (likewise y); the caller has checked the domain
__device__ __forceinline__ float bilinear(const Level& I, float x, float y) {
  const int ix = min((int)floorf(x), I.w - 2), iy = min((int)floorf(y), I.h - 2);
  const float fx = x - (float)ix, fy = y - (float)iy;
  const uint32_t o = (uint32_t)(iy * I.pitch + ix);
  const uint32_t r0 = ld16(I.p, o), r1 = ld16(I.p, o + (uint32_t)I.pitch);
  const float a = (float)(r0 & 0xFFu), b = (float)(r0 >> 8), c = (float)(r1 & 0xFFu), d = (float)(r1 >> 8);
  return (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
}

// Template samples at (x, y): I(x, y) and the central differences
// (I(x+1, y) - I(x-1, y)) / 2, (I(x, y+1) - I(x, y-1)) / 2, all bilinear as
// above. The caller has checked that x +- 1 and y +- 1 lie in the domain, so
// floor(x) - 1 >= 0 and floor(y) - 1 >= 0. The five samples share the 4x4
// window from (floor(x) - 1, floor(y) - 1) and the fractions of (x, y). At
// x = W-2 exactly the right sample's clamped form (ix = W-2, fx = 1) equals
// this one (ix = W-1, fx = 0), and the window's last column (x = W) enters
// with weight 0; likewise y = H-2 and the window's last row (y = H): each
// level buffer has a guard row, so these reads stay inside it.
__device__ __forceinline__ void template_samples(const Level& I, float x, float y, float& i0, float& gx, float& gy) {
  const int fxi = (int)floorf(x), fyi = (int)floorf(y);
  const float fx = x - (float)fxi, fy = y - (float)fyi;
  const uint32_t o = (uint32_t)((fyi - 1) * I.pitch + (fxi - 1));
  const uint32_t pt = (uint32_t)I.pitch;
  const uint32_t w0 = ld32(I.p, o), w1 = ld32(I.p, o + pt), w2 = ld32(I.p, o + 2u * pt), w3 = ld32(I.p, o + 3u * pt);
  const float gfx = 1.f - fx, gfy = 1.f - fy;
  auto px = [](uint32_t w, int c) { return (float)((w >> (8 * c)) & 0xFFu); };
  auto h = [&](uint32_t w, int c) { return gfx * px(w, c) + fx * px(w, c + 1); };
  const float h01 = h(w0, 1), h10 = h(w1, 0), h11 = h(w1, 1), h12 = h(w1, 2);
  const float h20 = h(w2, 0), h21 = h(w2, 1), h22 = h(w2, 2), h31 = h(w3, 1);
  i0 = gfy * h11 + fy * h21;
  const float ixp = gfy * h12 + fy * h22, ixm = gfy * h10 + fy * h20;
  const float iyp = gfy * h21 + fy * h31, iym = gfy * h01 + fy * h11;
  gx = (ixp - ixm) * 0.5f;
  gy = (iyp - iym) * 0.5f;
}

// Camera descriptors are read-only while the tracker runs: read through the
// constant address space, a wave-uniform descriptor's fields come in with
// scalar loads.
typedef const __attribute__((address_space(4))) CamDesc* cdesc_k;

// level l of pyramid slot `slot` of camera `cd`
__device__ __forceinline__ Level level_of(cdesc_k cd, int slot, int l) {
  Level L;
  L.p = (gbytes)cd->lvl[slot][l];
  L.pitch = cd->pitch[l];
  L.w = cd->w >> l;
  L.h = cd->h >> l;
  return L;
}

// A pointer every lane holds the same value of, marked so for the compiler
// (its loads then go through the scalar cache into scalar registers).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Sums of K values per level (level-major v[K*l + k]) over the first nl of L
// levels: all L levels in one call when all are used (the plain budget), else
// two levels at a time behind wave-uniform tests, so a short learned budget
// does not reduce the levels it never visits.
template <int L, int K, int l = 0>
__device__ __forceinline__ void level_pair_sums(float* v, int nl, int lane) {
  if constexpr (l < L) {
    if (l < nl) wave_sums<(l + 1 < L ? 2 : 1) * K>(v + K * l, lane);
    level_pair_sums<L, K, l + 2>(v, nl, lane);
  }
}
template <int L, int K>
__device__ __forceinline__ void level_sums(float* v, int nl, int lane) {
  if (nl >= L) wave_sums<K * L>(v, lane);
  else level_pair_sums<L, K>(v, nl, lane);
}

struct PassOut {
  int status;
  float tx, ty, th, resid;
};

// SE(2) exponential of (d0, d1, phi): translation V(phi) (d0, d1) with
// V = [[a, -b], [b, a]], a = sin(phi)/phi, b = (1 - cos(phi))/phi.
__device__ __forceinline__ void se2_v(float phi, float& a, float& b) {
  const float p2 = phi * phi;
  if (fabsf(phi) < 0.25f) {  // series, error below 2e-9 here
    a = 1.f - p2 * (1.f / 6.f - p2 * (1.f / 120.f - p2 * (1.f / 5040.f)));
    b = phi * (0.5f - p2 * (1.f / 24.f - p2 * (1.f / 720.f - p2 * (1.f / 40320.f))));
  } else {
    const float ip = rcp(phi);
    a = __sinf(phi) * ip;
    b = (1.f - __cosf(phi)) * ip;
  }
}

// One coarse-to-fine pass over the first nl <= L levels: template on `src` at
// (px, py), warp from (ix, iy, ith) (level-0 pixels), N Gauss-Newton
// iterations per level, levels nl-1 .. 0, translation doubled between levels,
// a level whose template does not fit is skipped.
template <int L>
__device__ __forceinline__ PassOut klt_pass(const CamDesc& csrc_in, int ssrc_in, const CamDesc& cdst_in, int sdst_in,
                                            float px, float py, float ix, float iy, float ith, int nl, int N, float u,
                                            float v, float wgt, int lane) {
  // the pass's cameras and slots are the wave's (the passes swap them)
  const cdesc_k csrc = (cdesc_k)uniform_ptr(&csrc_in);
  const cdesc_k cdst = (cdesc_k)uniform_ptr(&cdst_in);
  const int ssrc = __builtin_amdgcn_readfirstlane(ssrc_in), sdst = __builtin_amdgcn_readfirstlane(sdst_in);
  PassOut o{VIO_TRACKED, 0.f, 0.f, 0.f, 0.f};
  // ---- templates of all levels (Sec. III-E) ------------------------------
  bool fits[L], valid[L];
  float T[L], G0[L], G1[L], G2[L], k[3 * L];
  float I0[L], gxr[L], gyr[L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    fits[l] = false;
    I0[l] = gxr[l] = gyr[l] = 0.f;
    if (l < nl) {
      const Level S = level_of(csrc, ssrc, l);
      const float sc = 1.f / (float)(1 << l);
      const float sx = px * sc + u, sy = py * sc + v;
      fits[l] = wave_all(in_dom(S, sx - 1.f, sy) & in_dom(S, sx + 1.f, sy) & in_dom(S, sx, sy - 1.f) &
                         in_dom(S, sx, sy + 1.f));
      if (fits[l]) template_samples(S, sx, sy, I0[l], gxr[l], gyr[l]);
    }
  }
  float mean[L];
#pragma unroll
  for (int l = 0; l < L; ++l) mean[l] = wgt * I0[l];
  level_sums<L, 1>(mean, nl, lane);
  float J0[L], J1[L], J2[L], hs[6 * L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    mean[l] *= 1.f / 52.f;
    const float im = rcp(mean[l]);
    T[l] = I0[l] * im;
    J0[l] = gxr[l] * im;
    J1[l] = gyr[l] * im;
    J2[l] = J1[l] * u - J0[l] * v;
    hs[6 * l + 0] = wgt * J0[l] * J0[l];
    hs[6 * l + 1] = wgt * J0[l] * J1[l];
    hs[6 * l + 2] = wgt * J0[l] * J2[l];
    hs[6 * l + 3] = wgt * J1[l] * J1[l];
    hs[6 * l + 4] = wgt * J1[l] * J2[l];
    hs[6 * l + 5] = wgt * J2[l] * J2[l];
  }
  level_sums<L, 6>(hs, nl, lane);
#pragma unroll
  for (int l = 0; l < L; ++l) {
    valid[l] = false;
    k[3 * l + 0] = k[3 * l + 1] = k[3 * l + 2] = 0.f;
    G0[l] = G1[l] = G2[l] = 0.f;
    if (l >= nl) continue;  // a level the pass does not visit
    const float h00 = hs[6 * l + 0], h01 = hs[6 * l + 1], h02 = hs[6 * l + 2];
    const float h11 = hs[6 * l + 3], h12 = hs[6 * l + 4], h22 = hs[6 * l + 5];
    // 3x3 inverse by cofactors (H symmetric); degenerate when det <= 1e-6 (tr/3)^3
    const float c00 = h11 * h22 - h12 * h12;
    const float c01 = h12 * h02 - h01 * h22;
    const float c02 = h01 * h12 - h11 * h02;
    const float det = h00 * c00 + h01 * c01 + h02 * c02;
    const float tr3 = (h00 + h11 + h22) * (1.f / 3.f);
    const float id = rcp(det);
    const float i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    const float i11 = (h00 * h22 - h02 * h02) * id;
    const float i12 = (h02 * h01 - h00 * h12) * id;
    const float i22 = (h00 * h11 - h01 * h01) * id;
    // weight folded into the gains: lanes 52..63 contribute nothing
    G0[l] = wgt * (i00 * J0[l] + i01 * J1[l] + i02 * J2[l]);
    G1[l] = wgt * (i01 * J0[l] + i11 * J1[l] + i12 * J2[l]);
    G2[l] = wgt * (i02 * J0[l] + i12 * J1[l] + i22 * J2[l]);
    valid[l] = mean[l] > 0.f && det > 1e-6f * tr3 * tr3 * tr3 &&
               wave_all(isfinite(G0[l]) & isfinite(G1[l]) & isfinite(G2[l]));
    k[3 * l + 0] = G0[l] * T[l];
    k[3 * l + 1] = G1[l] * T[l];
    k[3 * l + 2] = G2[l] * T[l];
  }
  level_sums<L, 3>(k, nl, lane);
  // ---- coarse-to-fine Gauss-Newton (eqs. 4-5) ------------------------------
  float tx = ldexpf(ix, 1 - nl), ty = ldexpf(iy, 1 - nl), th = ith;
#pragma unroll
  for (int l = L - 1; l >= 0; --l) {
    if (l >= nl) continue;
    if (l < nl - 1) {
      tx = tx * 2.f;
      ty = ty * 2.f;
    }
    if (!fits[l]) {
      if (l == 0) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      continue;
    }
    if (!valid[l]) {
      o.status = VIO_LOST_DEGENERATE;
      return o;
    }
    const Level D = level_of(cdst, sdst, l);
    for (int it = 0; it < N; ++it) {
      const float cs = __cosf(th), sn = __sinf(th);
      const float wx = (cs * u - sn * v) + tx, wy = (sn * u + cs * v) + ty;
      if (wave_any(!in_dom(D, wx, wy))) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      const float Iw = bilinear(D, wx, wy);
      float S[4] = {wgt * Iw, G0[l] * Iw, G1[l] * Iw, G2[l] * Iw};
      wave_sums<4>(S, lane);
      const float mw = S[0] * (1.f / 52.f);
      if (!(mw > 0.f)) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      const float imw = rcp(mw);
      if (l == 0 && it == N - 1) {
        const float e = Iw * imw - T[l];
        o.resid = sqrtf(wave_sum(wgt * e * e, lane) * (1.f / 52.f));
      }
      const float d0 = k[3 * l + 0] - S[1] * imw, d1 = k[3 * l + 1] - S[2] * imw, d2 = k[3 * l + 2] - S[3] * imw;
      float a, b;
      se2_v(d2, a, b);
      const float vx = a * d0 - b * d1, vy = b * d0 + a * d1;
      tx = tx + (cs * vx - sn * vy);
      ty = ty + (sn * vx + cs * vy);
      th = th + d2;
    }
  }
  o.tx = tx;
  o.ty = ty;
  o.th = th;
  return o;
}

// ---- camera models of the camera-model start (Sec. III-E) ------------------
// A model is K = (fx, fy, cx, cy) plus, for the Kannala-Brandt equidistant
// fisheye (kb4 != 0), the coefficients k of its radius polynomial
// theta (1 + k0 theta^2 + k1 theta^4 + k2 theta^6 + k3 theta^8).
struct Model {
  const float* K;
  const float* k;
  int kb4;
};

__device__ __forceinline__ float kb4_radius(const float* k, float th, float& slope) {
  const float t2 = th * th;
  slope = 1.f + t2 * (3.f * k[0] + t2 * (5.f * k[1] + t2 * (7.f * k[2] + t2 * 9.f * k[3])));
  return th * (1.f + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3]))));
}

// rho times the point at inverse depth rho on pixel (x, y)'s ray: (a, b, 1)
// for the pinhole model, the unit ray for KB4 (the polynomial inverted by
// Newton's method from theta = theta_d; false without a root in [0, pi) where
// the radius rises with slope >= kKb4MinSlope: nearer the polynomial's fold
// the ray is ill-conditioned, and Newton's steps in FP32 stall at the root's
// resolution)
constexpr float kKb4MinSlope = 0.05f;
__device__ __forceinline__ bool model_ray(const Model& m, float x, float y, float X[3]) {
  const float a = (x - m.K[2]) / m.K[0], b = (y - m.K[3]) / m.K[1];
  if (!m.kb4) {
    X[0] = a;
    X[1] = b;
    X[2] = 1.f;
    return true;
  }
  const float td = sqrtf(a * a + b * b);
  float th = td, slope = 1.f;
  bool ok = true;
  // at most 12 steps (from theta_d, a root of slope >= kKb4MinSlope takes at
  // most 7); a step below 1e-6 (1 + theta) leaves an error of its square's
  // order, beneath FP32 resolution, so the loop ends there (every lane holds
  // the item's values, so the exit is wave-uniform)
#pragma unroll 1
  for (int it = 0; it < 12; ++it) {
    const float f = kb4_radius(m.k, th, slope) - td;
    ok &= slope > 0.f;
    const float step = ok ? f / slope : 0.f;
    th -= step;
    if (!(fabsf(step) > 1e-6f * (1.f + th))) break;
  }
  const float res = kb4_radius(m.k, th, slope) - td;
  // the residual of a converged root is at FP32 resolution: a few ulps of td
  if (!ok || !(slope >= kKb4MinSlope) || !(th >= 0.f) || !(th < 3.14159265f) || !(fabsf(res) <= 4e-6f * (1.f + td)))
    return false;
  const float sc = td > 0.f ? sinf(th) / td : 1.f;
  X[0] = sc * a;
  X[1] = sc * b;
  X[2] = cosf(th);
  return true;
}

// pixel of rho X (scaled as model_ray's); false for a pinhole point with
// rho Z <= 1e-6 and for a KB4 point on the axis behind the camera
__device__ __forceinline__ bool model_project(const Model& m, const float X[3], float& u, float& v) {
  if (!m.kb4) {
    if (!(X[2] > 1e-6f)) return false;
    u = m.K[0] * (X[0] / X[2]) + m.K[2];
    v = m.K[1] * (X[1] / X[2]) + m.K[3];
    return true;
  }
  const float r = sqrtf(X[0] * X[0] + X[1] * X[1]);
  if (!(r > 0.f)) {
    if (!(X[2] > 0.f)) return false;
    u = m.K[2];
    v = m.K[3];
    return true;
  }
  float slope;
  const float rd = kb4_radius(m.k, atan2f(r, X[2]), slope) / r;
  u = m.K[0] * (rd * X[0]) + m.K[2];
  v = m.K[1] * (rd * X[1]) + m.K[3];
  return true;
}

// (x, y) back-projected through `s` at inverse depth rho, moved by
// X' = R X + t, projected through `d`
__device__ __forceinline__ bool model_map(const Model& s, const Model& d, const float* R, const float* t, float rho,
                                          float x, float y, float& u, float& v) {
  float X[3], Y[3];
  if (!model_ray(s, x, y, X)) return false;
  for (int i = 0; i < 3; ++i) Y[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + rho * t[i];
  return model_project(d, Y, u, v);
}

// The start through any pair of models: the mapped pixel, and the angle of
// the mapped pixel step (1, 0) as the start rotation.
__device__ __forceinline__ bool model_start(const Model& s, const Model& d, const float* R, const float* t, float rho,
                                            float x, float y, float& ix, float& iy, float& ith) {
  float u0, v0, u1, v1;
  if (!model_map(s, d, R, t, rho, x, y, u0, v0) || !model_map(s, d, R, t, rho, x + 1.f, y, u1, v1)) return false;
  ix = u0;
  iy = v0;
  ith = atan2f(v1 - v0, u1 - u0);
  return true;
}

// Forward pass src -> dst from (ix, iy), then the backward pass dst -> src
// from the keypoint's own position, over nl levels with N iterations; both
// passes run the one inlined copy of the alignment code.
template <int L>
__device__ __forceinline__ TrackRes track_fb(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px,
                                             float py, float ix, float iy, float ith, int nl, int N, float fb_thr,
                                             float u, float v, float wgt, int lane) {
  TrackRes r;
  r.x = ix;
  r.y = iy;
  r.theta = 0.f;
  r.fb = 0.f;
  r.resid = 0.f;
  r.status = VIO_TRACKED;
  r.pad[0] = r.pad[1] = 0;
  const CamDesc* A = &csrc;
  const CamDesc* B = &cdst;
  int sa = ssrc, sb = sdst;
  float qx = px, qy = py, gx = ix, gy = iy, gth = ith;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const PassOut o = klt_pass<L>(*A, sa, *B, sb, qx, qy, gx, gy, gth, nl, N, u, v, wgt, lane);
    if (o.status != VIO_TRACKED) {
      r.status = o.status;
      break;
    }
    if (pass == 0) {
      r.x = o.tx;
      r.y = o.ty;
      r.theta = o.th;
      r.resid = o.resid;
      const CamDesc* t = A;
      A = B;
      B = t;
      const int st = sa;
      sa = sb;
      sb = st;
      qx = o.tx;
      qy = o.ty;
      gx = px;
      gy = py;
      gth = -o.th;
    } else {
      const float dx = o.tx - px, dy = o.ty - py;
      r.fb = sqrtf(dx * dx + dy * dy);
      r.status = r.fb > fb_thr ? VIO_LOST_FB : VIO_TRACKED;
    }
  }
  return r;
}

// Stores a wave-uniform 32-byte result without a branch on the lane id:
// lanes 0..7 write one dword each through a buffer resource whose range is
// exactly the record, and the hardware drops the other lanes' stores as out of
// range. (A lane-id branch inside the persistent loop would let the compiler
// split the wave across loop iterations; this keeps the loop body free of
// lane-dependent control flow.)
__device__ __forceinline__ void store_result(TrackRes* dst, const TrackRes& r, int lane) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)sizeof(TrackRes), kBufferWord3);
  const uint32_t w[8] = {__builtin_bit_cast(uint32_t, r.x),     __builtin_bit_cast(uint32_t, r.y),
                         __builtin_bit_cast(uint32_t, r.theta), __builtin_bit_cast(uint32_t, r.fb),
                         __builtin_bit_cast(uint32_t, r.resid), (uint32_t)r.status,
                         (uint32_t)r.pad[0],                    (uint32_t)r.pad[1]};
  uint32_t val = w[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) val = lane == k ? w[k] : val;
  __builtin_amdgcn_raw_buffer_store_b32(val, rs, lane * 4, 0, 0);
}

// The learned start of a temporal item when the learned stage is fused into
// the tracker: the keypoint's features -- the flows of the 8 nearest tracks
// with a flow in the previous frame's live set (exact keys; each lane reads
// its tracks straight from global memory in rising index order) and the
// pooled level-0 patch -- go to its feature row and, rounded to bfloat16, to
// the wave's LDS row; then the network runs on that row. The arithmetic is the
// learned-stage kernel's, so features and outputs are bit-identical to it.
// Loads are issued in the order they are needed (the patch and the first 512
// tracks, then half the weights, the rest after the search), so each wait
// covers only what it uses and the weights arrive during the search.
constexpr int kLearnCand = 8;  // tracks per lane loaded ahead of the search
__device__ __forceinline__ void learned_guess(const CamDesc& cd, const FrameCam& fc, const Kp* __restrict__ live,
                                              int n, int j, float kx, float ky, const Tuning& tune,
                                              uint16_t* sx, int lane, float out[3]) {
  int px4[4];
  patch_load(cd.lvl[fc.pyr_prev][0], cd.pitch[0], cd.w, cd.h, kx, ky, lane, true, px4);
  const double mx = (double)kx, my = (double)ky;
  float2 e[kLearnCand];
  int age[kLearnCand];
#pragma unroll
  for (int u = 0; u < kLearnCand; ++u) {
    const int k = u * kW + lane;
    e[u] = make_float2(0.f, 0.f);
    age[u] = 0;
    if (k < n) {
      e[u] = make_float2(live[k].x, live[k].y);
      age[u] = live[k].age;
    }
  }
  RowWeights W;
  W.load_first(tune.W1b, tune.W2b, lane);
  Top8 top;
  top.clear();
#pragma unroll
  for (int u = 0; u < kLearnCand; ++u) {
    const int k = u * kW + lane;
    if (k < n && age[u] >= 1) top.offer(e[u].x, e[u].y, mx, my, k);
  }
  for (int k = kLearnCand * kW + lane; k < n; k += kW) {  // more tracks than loaded ahead
    const Kp o = live[k];
    if (o.age >= 1) top.offer(o.x, o.y, mx, my, k);
  }
  W.load_second(tune.W2b, tune.W3b, lane);
  const int best = top.extract(lane);  // lane r < 8: the r-th nearest
  float* f = tune.feat + (size_t)(cd.row_off + j) * MI;
  if (lane < 8) {
    float fx = 0.f, fy = 0.f;
    if (best != kNone) {
      const Kp o = live[best];
      fx = (o.x - o.px) * 0.0625f;
      fy = (o.y - o.py) * 0.0625f;
    }
    reinterpret_cast<float2*>(f)[lane] = make_float2(fx, fy);
    sx[2 * lane] = bf16_bits(fx);
    sx[2 * lane + 1] = bf16_bits(fy);
  }
  float v;
  const int cell = patch_pool(px4, lane, v);
  if (cell >= 0) {
    f[16 + cell] = v;
    sx[16 + cell] = bf16_bits(v);
  }
  mlp_row(W, tune.mlpP, sx, sx + MI, lane, out);
}

// What one work item runs: cameras and pyramid slots, the keypoint, the
// starts and budgets of its attempts, and its record (out == nullptr: the item
// has nothing to do). Attempts first..last run, 0 the short budget from
// (gx, gy, gth), 1 the full one from (ix, iy, ith); a short track is kept when
// it passes the forward-backward check with a residual RMS <= srho.
struct Plan {
  const CamDesc* src;
  const CamDesc* dst;
  TrackRes* out;
  int ssrc, sdst;
  float px, py, ix, iy, ith, gx, gy, gth, srho;
  int sl, si, fl, fi;
  int first, last;
  int pad0;  // 1: a parallel fallback item, whose record always marks the fallback
};

// The plan of work item `item` (G = lanes per item: 64, or 32 with two items
// per wave, each half planning its own). A temporal track (camera c, slot j)
// starts from the caller's prediction, else from the camera-model projection
// when the frame carries a motion for the camera, else from the
// constant-velocity guess. Two tracks first try a short budget: with learned
// initialisation (tune.learned), an unpredicted track runs tune.llevels levels
// with tune.liters iterations from the network's guess, and a predicted one
// runs tune.plevels x tune.piters from its prediction when tune.plevels > 0.
// Otherwise, and whenever the short attempt does not hold, the full budget
// runs from the track's start (pad[0] = 1 marks such a fallback); a learned
// track's fallback from the constant-velocity start runs tune.fblevels x
// tune.fbiters. A stereo match of a detection (camera c, item j) starts from
// the rig's extrinsics when the target camera has them, else
// (tune.stereo_nb) from the nearest paired keypoint's offset with
// tune.slevels x tune.siters, else from the disparity prior with the full
// budget.
template <bool F, int G>
__device__ __forceinline__ Plan plan_item(const CamDesc* __restrict__ cams, const FrameTable* __restrict__ frame,
                                          const Counters* __restrict__ cnt, const TrackSeg* __restrict__ segs,
                                          int n_segs, const Prediction* __restrict__ pred, const Tuning& tune,
                                          int item, bool in_range, int lane, uint16_t* sx) {
  static_assert(G == kW || (G == kW / 2 && !F), "the fused learned stage runs one item per wave");
  Plan pl{};
  if (!in_range) return pl;
  // the last segment that begins at or before the item (begins ascend)
  int lo = 0, hi = n_segs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].begin <= item) lo = mid;
    else hi = mid - 1;
  }
  const TrackSeg sg = segs[lo];
  const int j = item - sg.begin;
  if (j < 0 || j >= sg.count) return pl;
  const int c = sg.cam;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active) return pl;
  const int P = fc.parity;
  pl.src = &cd;
  pl.ith = 0.f;
  // the budget of the attempt from (ix, iy, ith): the full one unless stated
  pl.fl = tune.levels;
  pl.fi = tune.iters;
  bool try_short = false;
  TrackRes* out;
  if (sg.mode != kModeStereo) {  // a temporal track, or its parallel fallback
    if (!fc.has_prev || j >= cnt->n_live[P ^ 1][c]) return pl;
    const Kp kp = cd.state[P ^ 1][j];
    pl.px = kp.x;
    pl.py = kp.y;
    pl.ix = kp.x + (kp.x - kp.px);
    pl.iy = kp.y + (kp.y - kp.py);
    bool predicted = false;
    const int np = fc.n_pred;
    if (np > 0) {  // caller predictions, ascending id: binary search
      const Prediction* pp = pred + fc.pred_off;
      int lo = 0, hi = np - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int64_t mid_id = pp[mid].id;
        if (mid_id == kp.id) {
          pl.ix = pp[mid].x;
          pl.iy = pp[mid].y;
          predicted = true;
          break;
        }
        if (mid_id < kp.id) lo = mid + 1;
        else hi = mid - 1;
      }
    }
    if (!predicted && fc.has_motion) {
      // camera-model start (Sec. III-E): back-project at inverse depth rho,
      // move by (R, t), project. With (a, b) = ((p - c) / f), rho X' =
      // R (a, b, 1) + rho t; the start rotation is the angle of
      // proj(p + (1, 0)) - proj(p), which in the same terms is
      // atan2((fy / fx) (R3 Z - R6 Y), R0 Z - R6 X) when both points lie in
      // front (Z, Z + R6 / fx > 0), without subtracting two projections.
      float rho = fc.rho;
      const int nd = fc.n_depth;
      if (nd > 0) {  // per-keypoint inverse depths, ascending id
        const KpDepth* dp = tune.depths + fc.depth_off;
        int lo = 0, hi = nd - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int64_t mid_id = dp[mid].id;
          if (mid_id == kp.id) {
            rho = dp[mid].rho;
            break;
          }
          if (mid_id < kp.id) lo = mid + 1;
          else hi = mid - 1;
        }
      }
      const float* R = fc.R;
      const float fx = fc.K[0], fy = fc.K[1];
      const float a = (kp.x - fc.K[2]) / fx, b = (kp.y - fc.K[3]) / fy;
      const float X = R[0] * a + R[1] * b + R[2] + rho * fc.t[0];
      const float Y = R[3] * a + R[4] * b + R[5] + rho * fc.t[1];
      const float Z = R[6] * a + R[7] * b + R[8] + rho * fc.t[2];
      if (fc.kb4) {
        const Model m{fc.K, fc.kk, 1};
        predicted = model_start(m, m, R, fc.t, rho, kp.x, kp.y, pl.ix, pl.iy, pl.ith);
      } else if (Z > 1e-6f && Z + R[6] / fx > 1e-6f) {
        pl.ix = fx * (X / Z) + fc.K[2];
        pl.iy = fy * (Y / Z) + fc.K[3];
        pl.ith = atan2f((fy / fx) * (R[3] * Z - R[6] * Y), R[0] * Z - R[6] * X);
        predicted = true;
      }
    }
    if (tune.learned && !predicted) {
      // the network's output: the learned stage's guess, or computed here when
      // the stage is fused (a parallel fallback item needs none)
      float gsv[3] = {0.f, 0.f, 0.f};
      if constexpr (F) {
        if (sg.mode != kModeFallback)
          learned_guess(cd, fc, cd.state[P ^ 1], __builtin_amdgcn_readfirstlane(cnt->n_live[P ^ 1][c]), j, kp.x,
                        kp.y, tune, sx, lane, gsv);
      } else {
        const float* gs = tune.guess + (size_t)(cd.row_off + j) * 3;
        gsv[0] = gs[0];
        gsv[1] = gs[1];
      }
      pl.gx = kp.x + 16.f * gsv[0];
      pl.gy = kp.y + 16.f * gsv[1];
      pl.sl = tune.llevels;
      pl.si = tune.liters;
      pl.srho = tune.rho;
      try_short = true;
      // the fallback from the constant-velocity start has its own budget
      pl.fl = tune.fblevels;
      pl.fi = tune.fbiters;
    }
    if (predicted && tune.plevels > 0) {
      // a predicted start needs a smaller search range: the short budget
      // first, the full one from the same start when it does not hold
      pl.gx = pl.ix;
      pl.gy = pl.iy;
      pl.gth = pl.ith;
      pl.sl = tune.plevels;
      pl.si = tune.piters;
      pl.srho = tune.prho;
      try_short = true;
    }
    pl.dst = &cd;
    pl.ssrc = fc.pyr_prev;
    pl.sdst = fc.pyr;
    out = cd.res + j;
    if (sg.mode == kModeFallback) {
      // the fallback attempt only, for a track that tries a short budget
      // first (its temporal item runs that, and the selection takes this
      // result when the short track is not kept)
      if (!try_short) return pl;
      pl.first = pl.last = 1;
      pl.pad0 = 1;
      pl.out = cd.res_fb + j;
      return pl;
    }
  } else {
    // stereo match of a detection into target camera c + 1 + t (item j =
    // t * nslots + i): speculative (i = the winner's key slot) or deferred
    // (i = the frame's i-th selected detection)
    const int t = cd.n_targets > 1 ? j / cd.nslots : 0;
    const int i = j - t * cd.nslots;
    if (tune.deferred) {
      if (i >= cnt->n_sel[c]) return pl;
      const Kp kp = cd.state[P][cnt->sel_base[c] + i];
      pl.px = kp.x;
      pl.py = kp.y;
    } else {
      const uint32_t key = cd.keys[fc.pyr][i];
      if (key == 0) return pl;
      const int idx = 0xFFFFFF - (int)(key & 0xFFFFFFu);
      pl.px = (float)(idx % cd.w);
      pl.py = (float)(idx / cd.w);
    }
    const float px = pl.px, py = pl.py;
    const int tc = c + 1 + t;
    const CamDesc* dst = &cams[tc];
    pl.dst = dst;
    pl.ix = px - tune.disparity0;
    pl.iy = py;
    if (tune.stereo_nb && !dst->has_ext) {
      // neighbour start: of the keypoints that after the previous frame lived
      // in both cameras (the target's pair table, id order), the nearest by
      // (squared distance in double, where the float differences and squares
      // are exact, then id) lends its offset; one candidate per lane per
      // round, then a minimum over the item's lanes
      const int Pq = frame->cam[tc].parity ^ 1;
      int np = cnt->n_pairs[Pq][tc];
      if constexpr (G == kW) np = __builtin_amdgcn_readfirstlane(np);  // wave-uniform trip count
      if (np > 0) {
        const float4* pt = dst->pairs[Pq];
        double bd = INFINITY;
        int bi = 0x7FFFFFFF;
        for (int q0 = 0; q0 < np; q0 += G) {
          const int q = q0 + (lane & (G - 1));
          if (q < np) {
            const float4 e = pt[q];
            const double dx = (double)e.x - (double)px, dy = (double)e.y - (double)py;
            const double d = dx * dx + dy * dy;
            if (d < bd) {  // q ascends per lane: an equal distance keeps the smaller index
              bd = d;
              bi = q;
            }
          }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
          const double od = __shfl_xor(bd, o);
          const int oi = __shfl_xor(bi, o);
          if (od < bd || (od == bd && oi < bi)) {
            bd = od;
            bi = oi;
          }
        }
        if constexpr (G == kW) bi = __builtin_amdgcn_readfirstlane(bi);
        const float4 e = pt[bi];
        pl.ix = px + e.z;
        pl.iy = py + e.w;
        pl.fl = tune.slevels;
        pl.fi = tune.siters;
      }
    }
    if (dst->has_ext) {
      // the rig's extrinsics (Sec. III-E's camera-model start): back-project
      // through the detecting camera at the default inverse depth, move,
      // project through the target camera; the rotation in closed form as for
      // the temporal start, with the two cameras' focal lengths
      const float* R = dst->ext_R;
      const float* Ks = dst->ext_Ks;
      const float* Kt = dst->ext_Kt;
      const float rho = dst->ext_rho;
      const float a = (px - Ks[2]) / Ks[0], b = (py - Ks[3]) / Ks[1];
      const float X = R[0] * a + R[1] * b + R[2] + rho * dst->ext_t[0];
      const float Y = R[3] * a + R[4] * b + R[5] + rho * dst->ext_t[1];
      const float Z = R[6] * a + R[7] * b + R[8] + rho * dst->ext_t[2];
      if (dst->ext_kbs || dst->ext_kbt) {
        const Model ms{Ks, dst->ext_ks, dst->ext_kbs}, mt{Kt, dst->ext_kt, dst->ext_kbt};
        float sx, sy, sth;
        if (model_start(ms, mt, R, dst->ext_t, rho, px, py, sx, sy, sth)) {
          pl.ix = sx;
          pl.iy = sy;
          pl.ith = sth;
        }
      } else if (Z > 1e-6f && Z + R[6] / Ks[0] > 1e-6f) {
        pl.ix = Kt[0] * (X / Z) + Kt[2];
        pl.iy = Kt[1] * (Y / Z) + Kt[3];
        pl.ith = atan2f(Kt[1] * (R[3] * Z - R[6] * Y), Kt[0] * (R[0] * Z - R[6] * X));
      }
    }
    pl.ssrc = fc.pyr;
    pl.sdst = fc.pyr;
    out = cd.sres + j;
  }
  // with parallel fallbacks a short attempt is the item's only one
  pl.first = try_short ? 0 : 1;
  pl.last = try_short && tune.par_fb ? 0 : 1;
  pl.out = out;
  return pl;
}

// One work item per wave.
template <int L, bool F>
__device__ __forceinline__ void process_item(const CamDesc* __restrict__ cams, const FrameTable* __restrict__ frame,
                                             const Counters* __restrict__ cnt, const TrackSeg* __restrict__ segs,
                                             int n_segs, const Prediction* __restrict__ pred, const Tuning& tune,
                                             int item, int lane, float u, float v, float wgt, uint16_t* sx) {
  const Plan pl = plan_item<F, kW>(cams, frame, cnt, segs, n_segs, pred, tune, item, true, lane, sx);
  if (!pl.out) return;
  TrackRes r;
  int fell_back = pl.pad0;
#pragma unroll 1
  for (int a = pl.first; a <= pl.last; ++a) {
    const bool short_run = a == 0;
    r = track_fb<L>(*pl.src, pl.ssrc, *pl.dst, pl.sdst, pl.px, pl.py, short_run ? pl.gx : pl.ix,
                    short_run ? pl.gy : pl.iy, short_run ? pl.gth : pl.ith, short_run ? pl.sl : pl.fl,
                    short_run ? pl.si : pl.fi, tune.fb_threshold, u, v, wgt, lane);
    if (short_run) {
      if (r.status == VIO_TRACKED && r.resid <= pl.srho) break;
      fell_back = 1;
    }
  }
  r.pad[0] = fell_back;
  store_result(pl.out, r, lane);
}

// ---- two keypoints per wave -------------------------------------------------
// Half h = lane / 32 of the wave tracks one keypoint; lane g = lane mod 32 of a
// half holds pattern points g (index 0 of the per-lane arrays) and g + 32
// (index 1; weight 0 from g = 20 on, where the index passes the 52 points).
// Per keypoint the steps, decisions and arithmetic are those of klt_pass, and
// the sums over the pattern run through the same tree (half_sums), so a half
// computes what one wave computes for the same keypoint, bit for bit. Levels,
// iterations and descriptors are the wave's; `act` (uniform across each half)
// says which halves run the pass. A half that leaves the procedure keeps its
// status and idles (its loads masked off) while the other half goes on.
// level_sums for two keypoints per wave: out[K l + k] <- the half's total of
// value k of level l, gen(K l + k, point) giving each lane's two values.
template <int L, int K, int l = 0, class Gen>
__device__ __forceinline__ void level_pair_sums2(float* out, const Gen& gen, int nl, int lane) {
  if constexpr (l < L) {
    if (l < nl) half_sums_of<(l + 1 < L ? 2 : 1) * K, K * l>(out, gen, lane);
    level_pair_sums2<L, K, l + 2>(out, gen, nl, lane);
  }
}
template <int L, int K, class Gen>
__device__ __forceinline__ void level_sums2(float* out, const Gen& gen, int nl, int lane) {
  if (nl >= L) half_sums_of<K * L, 0>(out, gen, lane);
  else level_pair_sums2<L, K>(out, gen, nl, lane);
}

template <int L>
__device__ __forceinline__ PassOut klt_pass2(const CamDesc& csrc_in, int ssrc_in, const CamDesc& cdst_in, int sdst_in,
                                             float px, float py, float ix, float iy, float ith, int nl_in, int N_in,
                                             const float* u, const float* v, float wb, bool act, int lane) {
  // point g < 32 is always one of the 52: its weight is 1
  const float wgt[2] = {1.f, wb};
  const cdesc_k csrc = (cdesc_k)uniform_ptr(&csrc_in);
  const cdesc_k cdst = (cdesc_k)uniform_ptr(&cdst_in);
  const int ssrc = __builtin_amdgcn_readfirstlane(ssrc_in), sdst = __builtin_amdgcn_readfirstlane(sdst_in);
  const int nl = __builtin_amdgcn_readfirstlane(nl_in), N = __builtin_amdgcn_readfirstlane(N_in);
  PassOut o{VIO_TRACKED, 0.f, 0.f, 0.f, 0.f};
  bool live = act;  // the half is still in the procedure
  // ---- templates of all levels (Sec. III-E) ------------------------------
  bool fits[L], valid[L];
  float T[L][2], G0[L][2], G1[L][2], G2[L][2], k[3 * L];
  float I0[L][2], gxr[L][2], gyr[L][2];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    fits[l] = false;
#pragma unroll
    for (int q = 0; q < 2; ++q) I0[l][q] = gxr[l][q] = gyr[l][q] = 0.f;
    if (l < nl) {
      const Level S = level_of(csrc, ssrc, l);
      const float sc = 1.f / (float)(1 << l);
      float sx[2], sy[2];
      bool in = true;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        sx[q] = px * sc + u[q];
        sy[q] = py * sc + v[q];
        in = in & in_dom(S, sx[q] - 1.f, sy[q]) & in_dom(S, sx[q] + 1.f, sy[q]) & in_dom(S, sx[q], sy[q] - 1.f) &
             in_dom(S, sx[q], sy[q] + 1.f);
      }
      fits[l] = half_all(in, lane) && live;
      if (fits[l]) {
#pragma unroll
        for (int q = 0; q < 2; ++q) template_samples(S, sx[q], sy[q], I0[l][q], gxr[l][q], gyr[l][q]);
      }
    }
  }
  float mean[L];
  level_sums2<L, 1>(mean, [&](int l, int q) { return wgt[q] * I0[l][q]; }, nl, lane);
  float J0[L][2], J1[L][2], J2[L][2];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    mean[l] *= 1.f / 52.f;
    const float im = rcp(mean[l]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T[l][q] = I0[l][q] * im;
      J0[l][q] = gxr[l][q] * im;
      J1[l][q] = gyr[l][q] * im;
      J2[l][q] = J1[l][q] * u[q] - J0[l][q] * v[q];
    }
  }
  // H_l = sum w J^T J: (00, 01, 02, 11, 12, 22) of level l at 6 l .. 6 l + 5
  float hs[6 * L];
  level_sums2<L, 6>(
      hs,
      [&](int i, int q) {
        const int l = i / 6, m = i % 6;
        const float a = m < 3 ? J0[l][q] : m < 5 ? J1[l][q] : J2[l][q];
        const float b = m == 0 ? J0[l][q] : m == 1 || m == 3 ? J1[l][q] : J2[l][q];
        return wgt[q] * a * b;
      },
      nl, lane);
#pragma unroll
  for (int l = 0; l < L; ++l) {
    valid[l] = false;
#pragma unroll
    for (int q = 0; q < 2; ++q) G0[l][q] = G1[l][q] = G2[l][q] = 0.f;
    if (l >= nl) continue;  // a level the pass does not visit
    const float h00 = hs[6 * l + 0], h01 = hs[6 * l + 1], h02 = hs[6 * l + 2];
    const float h11 = hs[6 * l + 3], h12 = hs[6 * l + 4], h22 = hs[6 * l + 5];
    // 3x3 inverse by cofactors (H symmetric); degenerate when det <= 1e-6 (tr/3)^3
    const float c00 = h11 * h22 - h12 * h12;
    const float c01 = h12 * h02 - h01 * h22;
    const float c02 = h01 * h12 - h11 * h02;
    const float det = h00 * c00 + h01 * c01 + h02 * c02;
    const float tr3 = (h00 + h11 + h22) * (1.f / 3.f);
    const float id = rcp(det);
    const float i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    const float i11 = (h00 * h22 - h02 * h02) * id;
    const float i12 = (h02 * h01 - h00 * h12) * id;
    const float i22 = (h00 * h11 - h01 * h01) * id;
    bool fin = true;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      G0[l][q] = wgt[q] * (i00 * J0[l][q] + i01 * J1[l][q] + i02 * J2[l][q]);
      G1[l][q] = wgt[q] * (i01 * J0[l][q] + i11 * J1[l][q] + i12 * J2[l][q]);
      G2[l][q] = wgt[q] * (i02 * J0[l][q] + i12 * J1[l][q] + i22 * J2[l][q]);
      fin = fin & isfinite(G0[l][q]) & isfinite(G1[l][q]) & isfinite(G2[l][q]);
    }
    valid[l] = mean[l] > 0.f && det > 1e-6f * tr3 * tr3 * tr3 && half_all(fin, lane);
  }
  // c_l = sum G_i T_i
  level_sums2<L, 3>(
      k,
      [&](int i, int q) {
        const int l = i / 3, m = i % 3;
        return (m == 0 ? G0[l][q] : m == 1 ? G1[l][q] : G2[l][q]) * T[l][q];
      },
      nl, lane);
  // ---- coarse-to-fine Gauss-Newton (eqs. 4-5) ------------------------------
  float tx = ldexpf(ix, 1 - nl), ty = ldexpf(iy, 1 - nl), th = ith;
#pragma unroll
  for (int l = L - 1; l >= 0; --l) {
    if (l >= nl) continue;
    if (l < nl - 1) {
      tx = tx * 2.f;
      ty = ty * 2.f;
    }
    // a level whose template does not fit is skipped, and at level 0 the track is lost
    if (live && !fits[l] && l == 0) {
      o.status = VIO_LOST_OOB;
      live = false;
    }
    if (live && fits[l] && !valid[l]) {
      o.status = VIO_LOST_DEGENERATE;
      live = false;
    }
    bool run = live && fits[l];
    if (!wave_any(run)) {
      if (!wave_any(live)) break;
      continue;
    }
    const Level D = level_of(cdst, sdst, l);
    for (int it = 0; it < N; ++it) {
      const float cs = __cosf(th), sn = __sinf(th);
      float wx[2], wy[2];
      bool in = true;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        wx[q] = (cs * u[q] - sn * v[q]) + tx;
        wy[q] = (sn * u[q] + cs * v[q]) + ty;
        in = in & in_dom(D, wx[q], wy[q]);
      }
      if (half_any(!in, lane) && run) {
        o.status = VIO_LOST_OOB;
        live = run = false;
      }
      if (!wave_any(run)) break;
      float Iw[2] = {0.f, 0.f};
      if (run) {
#pragma unroll
        for (int q = 0; q < 2; ++q) Iw[q] = bilinear(D, wx[q], wy[q]);
      }
      float S[4] = {wgt[0] * Iw[0], G0[l][0] * Iw[0], G1[l][0] * Iw[0], G2[l][0] * Iw[0]};
      const float Sb[4] = {wgt[1] * Iw[1], G0[l][1] * Iw[1], G1[l][1] * Iw[1], G2[l][1] * Iw[1]};
      half_sums<4>(S, Sb, lane);
      const float mw = S[0] * (1.f / 52.f);
      if (run && !(mw > 0.f)) {
        o.status = VIO_LOST_OOB;
        live = run = false;
      }
      const float imw = rcp(mw);
      if (l == 0 && it == N - 1) {
        const float e0 = Iw[0] * imw - T[l][0], e1 = Iw[1] * imw - T[l][1];
        const float rs = sqrtf(half_sum(wgt[0] * e0 * e0, wgt[1] * e1 * e1, lane) * (1.f / 52.f));
        if (run) o.resid = rs;
      }
      const float d0 = k[3 * l + 0] - S[1] * imw, d1 = k[3 * l + 1] - S[2] * imw, d2 = k[3 * l + 2] - S[3] * imw;
      float a, b;
      se2_v(d2, a, b);
      const float vx = a * d0 - b * d1, vy = b * d0 + a * d1;
      const float ntx = tx + (cs * vx - sn * vy);
      const float nty = ty + (sn * vx + cs * vy);
      const float nth = th + d2;
      if (run) {
        tx = ntx;
        ty = nty;
        th = nth;
      }
    }
    if (!wave_any(live)) break;
  }
  o.tx = tx;
  o.ty = ty;
  o.th = th;
  return o;
}

// track_fb for two keypoints per wave: the forward pass from (ix, iy, ith),
// then, for each half whose forward track holds, the backward pass from it.
template <int L>
__device__ __forceinline__ TrackRes track_fb2(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px,
                                              float py, float ix, float iy, float ith, int nl, int N, float fb_thr,
                                              const float* u, const float* v, float wb, bool act, int lane) {
  TrackRes r;
  r.x = ix;
  r.y = iy;
  r.theta = 0.f;
  r.fb = 0.f;
  r.resid = 0.f;
  r.status = VIO_TRACKED;
  r.pad[0] = r.pad[1] = 0;
  const CamDesc* A = &csrc;
  const CamDesc* B = &cdst;
  int sa = ssrc, sb = sdst;
  float qx = px, qy = py, gx = ix, gy = iy, gth = ith;
  bool run = act;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    if (!wave_any(run)) break;
    const PassOut o = klt_pass2<L>(*A, sa, *B, sb, qx, qy, gx, gy, gth, nl, N, u, v, wb, run, lane);
    const bool ok = run && o.status == VIO_TRACKED;
    if (run && !ok) r.status = o.status;
    if (pass == 0) {
      if (ok) {
        r.x = o.tx;
        r.y = o.ty;
        r.theta = o.th;
        r.resid = o.resid;
      }
      const CamDesc* t = A;
      A = B;
      B = t;
      const int st = sa;
      sa = sb;
      sb = st;
      qx = o.tx;
      qy = o.ty;
      gx = px;
      gy = py;
      gth = -o.th;
    } else if (ok) {
      const float dx = o.tx - px, dy = o.ty - py;
      r.fb = sqrtf(dx * dx + dy * dy);
      r.status = r.fb > fb_thr ? VIO_LOST_FB : VIO_TRACKED;
    }
    run = ok;
  }
  return r;
}

// A value of lane `src` (a wave-uniform constant) to every lane.
template <class T>
__device__ __forceinline__ T* lane_ptr(T* p, int src) {
  const uint64_t x = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int lane_int(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ __forceinline__ float lane_float(float x, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), src));
}

// store_result for two keypoints per wave: lanes 32h .. 32h + 7 write half h's
// record (dst of lane 32h; nullptr: none), the other lanes' stores fall
// outside each record's buffer range.
__device__ __forceinline__ void store_result2(TrackRes* dst, const TrackRes& r, int lane) {
  const uint32_t w[8] = {__builtin_bit_cast(uint32_t, r.x),     __builtin_bit_cast(uint32_t, r.y),
                         __builtin_bit_cast(uint32_t, r.theta), __builtin_bit_cast(uint32_t, r.fb),
                         __builtin_bit_cast(uint32_t, r.resid), (uint32_t)r.status,
                         (uint32_t)r.pad[0],                    (uint32_t)r.pad[1]};
  const int g = lane & 31;
  uint32_t val = w[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) val = g == k ? w[k] : val;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    TrackRes* d = lane_ptr(dst, 32 * h);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(d, (short)0, d ? (int)sizeof(TrackRes) : 0, kBufferWord3);
    __builtin_amdgcn_raw_buffer_store_b32(val, rs, (lane >> 5) == h ? g * 4 : 1024, 0, 0);
  }
}

// Two work items per wave, one per half (item_in_range: the half's item
// exists). Each half plans its item and parks the plan in the wave's LDS (two
// slots, sp), read back field by field where used, so the plan does not hold
// registers through the tracking. The attempts then run for both halves at
// once when they share cameras, pyramid slots and budget, else one half after
// the other (a pair that straddles two segments or two budgets).
template <int L>
__device__ __forceinline__ void process_pair(const CamDesc* __restrict__ cams, const FrameTable* __restrict__ frame,
                                             const Counters* __restrict__ cnt, const TrackSeg* __restrict__ segs,
                                             int n_segs, const Prediction* __restrict__ pred, const Tuning& tune,
                                             int item, bool item_in_range, int lane, const float* u, const float* v,
                                             float wb, Plan* sp) {
  {
    const Plan pl =
        plan_item<false, kW / 2>(cams, frame, cnt, segs, n_segs, pred, tune, item, item_in_range, lane, nullptr);
    if ((lane & 31) == 0) sp[lane >> 5] = pl;
    wave_sync_lds();
  }
  const Plan& me = sp[lane >> 5];
  const Plan& p0 = sp[0];
  const Plan& p1 = sp[1];
  TrackRes r{};
  int fell_back = me.pad0;
  bool done = false;
#pragma unroll 1
  for (int a = 0; a <= 1; ++a) {
    const bool want = me.out != nullptr && !done && me.first <= a && a <= me.last;
    if (!wave_any(want)) continue;
    const bool short_run = a == 0;
    const bool w0 = lane_int(want, 0) != 0, w1 = lane_int(want, 32) != 0;
    const bool same = w0 && w1 && p0.src == p1.src && p0.dst == p1.dst && p0.ssrc == p1.ssrc &&
                      p0.sdst == p1.sdst && (short_run ? p0.sl == p1.sl && p0.si == p1.si
                                                       : p0.fl == p1.fl && p0.fi == p1.fi);
    const int rounds = w0 && w1 && !same ? 2 : 1;
#pragma unroll 1
    for (int rd = 0; rd < rounds; ++rd) {
      const int hs = rd == 1 || !w0 ? 1 : 0;  // the half whose cameras, slots and budget the round takes
      const bool act = want && (same || (lane >> 5) == hs);
      const Plan& ph = sp[hs];
      const TrackRes t = track_fb2<L>(*ph.src, ph.ssrc, *ph.dst, ph.sdst, me.px, me.py, short_run ? me.gx : me.ix,
                                      short_run ? me.gy : me.iy, short_run ? me.gth : me.ith,
                                      short_run ? ph.sl : ph.fl, short_run ? ph.si : ph.fi, tune.fb_threshold, u, v,
                                      wb, act, lane);
      if (act) r = t;
    }
    if (short_run && want) {
      done = r.status == VIO_TRACKED && r.resid <= me.srho;
      if (!done) fell_back = 1;
    }
  }
  r.pad[0] = fell_back;
  store_result2(me.out, r, lane);
}

// One wave per work item. F: the learned stage is fused (each wave has a row
// of LDS for the network).
template <int L, bool F>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track(const CamDesc* __restrict__ cams,
                                                          const FrameTable* __restrict__ frame,
                                                          const Counters* __restrict__ cnt,
                                                          const TrackSeg* __restrict__ segs, int n_segs,
                                                          int item_base, int n_items,
                                                          const Prediction* __restrict__ pred, Tuning tune) {
  const int lane = threadIdx.x & (kW - 1);
  // the wave's item: uniform across the wave (readfirstlane tells the compiler
  // so, which keeps the item's descriptors and pyramid bases in scalar
  // registers, loaded through the scalar cache)
  const int k = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (int)(blockDim.x / kW) + (int)(threadIdx.x / kW));
  if (k >= n_items) return;
  uint16_t* sx = nullptr;
  if constexpr (F) {
    __shared__ __align__(16) uint16_t sLearn[kTrackWaves][MI + MH];
    sx = sLearn[threadIdx.x / kW];
  }
  float u, v, wgt;
  pattern_of(lane, u, v, wgt);
  process_item<L, F>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + k, lane, u, v, wgt, sx);
}

// Persistent grid: every wave pops items from the frame's queue counter until
// it runs past n_items (each pop advances the counter, so every wave exits).
// The pop is branch-free: all lanes issue the atomic, lane 0 adding one and
// the others zero, and the first lane's (lane 0's) old value is the item, so
// no lane-dependent control flow enters the loop.
template <int L, bool F>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track_persistent(const CamDesc* __restrict__ cams,
                                                                     FrameTable* __restrict__ frame,
                                                                     const Counters* __restrict__ cnt,
                                                                     const TrackSeg* __restrict__ segs, int n_segs,
                                                                     int item_base, int n_items,
                                                                     const Prediction* __restrict__ pred,
                                                                     Tuning tune, int queue) {
  const int lane = threadIdx.x & (kW - 1);
  uint16_t* sx = nullptr;
  if constexpr (F) {
    __shared__ __align__(16) uint16_t sLearn[kTrackWaves][MI + MH];
    sx = sLearn[threadIdx.x / kW];
  }
  float u, v, wgt;
  pattern_of(lane, u, v, wgt);
  for (;;) {
    const int k = __builtin_amdgcn_readfirstlane(atomicAdd(&frame->queue_head[queue], lane == 0 ? 1 : 0));
    if (k >= n_items) break;
    process_item<L, F>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + k, lane, u, v, wgt, sx);
  }
}

// Two work items per wave (the throughput shape for many items): wave k runs
// items 2k (half 0) and 2k + 1 (half 1).
template <int L>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track2(const CamDesc* __restrict__ cams,
                                                           const FrameTable* __restrict__ frame,
                                                           const Counters* __restrict__ cnt,
                                                           const TrackSeg* __restrict__ segs, int n_segs,
                                                           int item_base, int n_items,
                                                           const Prediction* __restrict__ pred, Tuning tune) {
  const int lane = threadIdx.x & (kW - 1);
  const int k = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (int)(blockDim.x / kW) + (int)(threadIdx.x / kW));
  if (2 * k >= n_items) return;
  __shared__ Plan sPlan[kTrackWaves][2];
  float u[2], v[2], w0, wb;
  pattern_of(lane & 31, u[0], v[0], w0);
  pattern_of((lane & 31) + 32, u[1], v[1], wb);
  const int it = 2 * k + (lane >> 5);
  process_pair<L>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + it, it < n_items, lane, u, v, wb,
                  sPlan[threadIdx.x / kW]);
}

// The persistent grid with two items per wave: each pop takes two items.
template <int L>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track2_persistent(const CamDesc* __restrict__ cams,
                                                                      FrameTable* __restrict__ frame,
                                                                      const Counters* __restrict__ cnt,
                                                                      const TrackSeg* __restrict__ segs, int n_segs,
                                                                      int item_base, int n_items,
                                                                      const Prediction* __restrict__ pred,
                                                                      Tuning tune, int queue) {
  const int lane = threadIdx.x & (kW - 1);
  __shared__ Plan sPlan[kTrackWaves][2];
  float u[2], v[2], w0, wb;
  pattern_of(lane & 31, u[0], v[0], w0);
  pattern_of((lane & 31) + 32, u[1], v[1], wb);
  for (;;) {
    const int k = __builtin_amdgcn_readfirstlane(atomicAdd(&frame->queue_head[queue], lane == 0 ? 2 : 0));
    if (k >= n_items) break;
    const int it = k + (lane >> 5);
    process_pair<L>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + it, it < n_items, lane, u, v, wb,
                    sPlan[threadIdx.x / kW]);
    wave_sync_lds();  // the next item's plan overwrites this one's
  }
}

template <int L, bool F>
hipError_t launch_LF(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                     int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape sh, hipStream_t s) {
  const int bw = sh.block_waves;
  const int item_waves = sh.kp_per_wave == 2 ? (n_items + 1) / 2 : n_items;
  if (sh.waves_per_cu > 0) {
    const int waves = std::min(item_waves, sh.waves_per_cu * sh.n_cus);
    const int blocks = (waves + bw - 1) / bw;
    if constexpr (!F) {
      if (sh.kp_per_wave == 2) {
        launch_kernel(k_track2_persistent<L>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs,
                      n_segs, item_base, n_items, d_pred, tune, sh.queue);
        return hipGetLastError();
      }
    }
    launch_kernel(k_track_persistent<L, F>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs,
                  n_segs, item_base, n_items, d_pred, tune, sh.queue);
  } else {
    const int blocks = (item_waves + bw - 1) / bw;
    if constexpr (!F) {
      if (sh.kp_per_wave == 2) {
        launch_kernel(k_track2<L>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs, n_segs,
                      item_base, n_items, d_pred, tune);
        return hipGetLastError();
      }
    }
    launch_kernel(k_track<L, F>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs, n_segs,
                  item_base, n_items, d_pred, tune);
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_L(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                    int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape sh, hipStream_t s) {
  if (tune.learned && tune.fused)
    return launch_LF<L, true>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
  return launch_LF<L, false>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
}

}  // namespace

hipError_t launch_track(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                        int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape shape,
                        hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (shape.block_waves < 1 || shape.block_waves > kTrackWaves || shape.n_cus < 1 || shape.waves_per_cu < 0 ||
      shape.queue < 0 || shape.queue >= 4 || (shape.kp_per_wave != 1 && shape.kp_per_wave != 2))
    return hipErrorInvalidValue;
  // the fused learned stage runs one item per wave
  if (shape.kp_per_wave == 2 && tune.learned && tune.fused) return hipErrorInvalidValue;
  // the short tracker of learned initialisation runs within the full one's levels
  if (tune.learned && (tune.llevels < 1 || tune.llevels > tune.levels || tune.liters < 1)) return hipErrorInvalidValue;
  switch (tune.levels) {
#define VIO_TRACK_CASE(LV) \
  case LV: return launch_L<LV>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, shape, s);
    VIO_TRACK_CASE(1)
    VIO_TRACK_CASE(2)
    VIO_TRACK_CASE(3)
    VIO_TRACK_CASE(4)
    VIO_TRACK_CASE(5)
    VIO_TRACK_CASE(6)
#undef VIO_TRACK_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vio
