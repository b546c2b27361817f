// Fused pyramid + corner detector for gfx950.
//
// One workgroup owns a TxT level-0 tile of one camera (T = 64 with 1024
// threads, or T = 32 with 256 threads: more, smaller workgroups for small
// images, chosen per workload at create). It stages
// the tile plus an apron in LDS with coalesced dword loads, then
//  * computes the FAST-9 score (Sec. III-D) of the tile and a one-pixel ring
//    (the paper's early rejection on ring pairs (0,8)/(4,12) over every pixel,
//    the survivors compacted into an LDS list, then the score over the list,
//    both polarities at once in 16-bit halves), keeps strict 3x3 maxima with
//    score >= the last threshold and folds each into its cell's packed
//    winner keys with atomicMax, and
//  * builds every coarser pyramid level of the tile (Sec. III-C, eqs. 2-3)
//    from LDS, recomputing the apron instead of reading it back from HBM, so
//    level 0 is read from HBM once per frame and the L-1 level-serial
//    dispatches of the paper become one launch.
// All arithmetic is integer, so the result is bit-identical to a level-serial
// build.
//
// Threshold walk (Sec. III-D): walking the decreasing thresholds 40, 20, 10, 5
// and stopping at the first level with k survivors in the cell keeps the same
// top k as one pass at the last threshold. A strict local maximum does not
// depend on the threshold (a neighbour below it scores less than the candidate
// anyway), so the survivor sets of the levels are nested, and whenever some
// level holds k of them its top k are the top k of the last level's set. The
// cell's winners are its largest keys
// key = score << 24 | (2^24 - 1 - (y * W + x)), i.e. highest score, then
// smallest y, then smallest x: one atomicMax per survivor for k = 1, a chain
// of k max-exchange slots otherwise.
#include "fe_common.h"
#include "wave_ops.h"

namespace vio {
namespace {

template <int L, int T>
struct PyrGeom {
  static constexpr int threads = T == 64 ? 1024 : 256;
  static constexpr int score_edge = T + 2;
  // apron of level l so that the tile of level L-1 can be computed: A[L-1] = 0,
  // A[l] = 2 A[l+1] + 2, i.e. A[l] = 2^(L-l) - 2
  static constexpr __host__ __device__ int apron(int l) { return (1 << (L - l)) - 2; }
  static constexpr __host__ __device__ int tile(int l) { return T >> l; }
  static constexpr __host__ __device__ int region(int l) { return tile(l) + 2 * apron(l); }
  // level-0 staging: apron at least 4 (FAST radius 3 plus the NMS ring)
  static constexpr int a0 = apron(0) > 4 ? apron(0) : 4;
  static constexpr int a0x = (a0 + 3) & ~3;  // left apron rounded to a dword
  // the early rejection tests four pixels at a time: group g holds score-region
  // columns 4g-3 .. 4g (dword-aligned in LDS), and reads the dwords on either
  // side of its middle row
  static constexpr int fast_groups = (score_edge + 2) / 4 + 1;
  static constexpr int sw0_min = ((T + a0x + a0) + 3) & ~3;
  static constexpr int sw0 = sw0_min > 4 * fast_groups + a0x ? sw0_min : 4 * fast_groups + a0x;
  static constexpr int score_bytes = (score_edge * score_edge + 3) & ~3;
  static constexpr int sh0 = T + 2 * a0;
  static constexpr int vbytes = L > 1 ? (region(0) - 1) * region(1) : 1;
  // the paired horizontal pass reads three dwords from byte 4q of a level-0
  // row: bytes up to 2 region(1) + 7 stay inside the staged row
  static_assert(L == 1 || 2 * region(1) + 8 <= sw0, "staged level-0 row too short for the paired pass");
  // byte offset of input column 2 o_x - 2 (o_x: level-1 region origin) in
  // its dword of a staged level-0 row; above level 0 the region origins nest
  // and the offset is 0
  static constexpr int h_shift0 = a0x - apron(0);
  static_assert(L == 1 || (h_shift0 >= 0 && h_shift0 < 4), "paired pass byte shift");
  static constexpr int lvl_bytes = L > 1 ? region(1) * region(1) : 1;
  // tiles per XCD run: 512 level-0 pixels
  static constexpr int xcd_run = 512 / T;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Tile of workgroup b among n. Workgroups go to the 8 XCDs in turn (b mod 8),
// each XCD with its own L2, and a staged row (tile plus aprons) spans two
// 128-byte lines that the horizontal neighbours share: with tiles in raster
// order every neighbour sits on another XCD and each L2 fetches the shared
// lines again. Here XCD x takes runs of R consecutive tiles (workgroups x,
// x + 8, x + 16, ... take run x, then run x + 8, ...), so a run's shared lines
// are fetched once into one L2, while the runs still interleave finely over
// the XCDs (no band of the image lands on one XCD). Workgroups past the last
// whole group of 8 runs keep their own index. A permutation of 0..n-1.
constexpr int kXcds = 8;
template <int R>
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int group = kXcds * R;
  if (b >= n / group * group) return b;
  const int x = b % kXcds, j = b / kXcds;
  return ((j / R) * kXcds + x) * R + j % R;
}

// Signed differences of the 16 circle pixels to the centre (Bresenham circle
// of radius 3 from (0,-3) clockwise), read from the LDS tile at offset `o`
// with row pitch `sp`.
__device__ __forceinline__ void ring_diffs(const uint8_t* img, int o, int sp, int d[16]) {
  const int c = img[o];
  d[0] = img[o - 3 * sp] - c;
  d[1] = img[o - 3 * sp + 1] - c;
  d[2] = img[o - 2 * sp + 2] - c;
  d[3] = img[o - sp + 3] - c;
  d[4] = img[o + 3] - c;
  d[5] = img[o + sp + 3] - c;
  d[6] = img[o + 2 * sp + 2] - c;
  d[7] = img[o + 3 * sp + 1] - c;
  d[8] = img[o + 3 * sp] - c;
  d[9] = img[o + 3 * sp - 1] - c;
  d[10] = img[o + 2 * sp - 2] - c;
  d[11] = img[o + sp - 3] - c;
  d[12] = img[o - 3] - c;
  d[13] = img[o - sp - 3] - c;
  d[14] = img[o - 2 * sp - 2] - c;
  d[15] = img[o - 3 * sp - 1] - c;
}

typedef short short2v __attribute__((ext_vector_type(2)));

// The paper's early rejection (Sec. III-D): every 9-arc holds one of the ring
// positions 0 and 8 and one of 4 and 12, so a corner at threshold tmin needs
// such a pair brighter than I(p) + tmin or darker than I(p) - tmin, i.e.
//   min(max(p0, p8), max(p4, p12)) - I(p) > tmin   (bright) or
//   I(p) - max(min(p0, p8), min(p4, p12)) > tmin   (dark).
// Four horizontally adjacent pixels at once: byte k of c is pixel k, of p0,
// p4, p8, p12 its ring pixels 0 (above), 4 (right), 8 (below), 12 (left);
// bytes 0, 2 and then 1, 3 ride in 16-bit halves. Bit k of the result is set
// when pixel k passes.
__device__ __forceinline__ uint32_t fast_may_pass4(uint32_t p0, uint32_t p4, uint32_t p8, uint32_t p12, uint32_t c,
                                                   int tmin) {
  const short2v tm = {(short)tmin, (short)tmin};
  uint32_t res = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    auto pair = [h](uint32_t w) { return __builtin_bit_cast(short2v, (w >> (8 * h)) & 0x00FF00FFu); };
    const short2v a = pair(p0), b = pair(p8), r = pair(p4), l = pair(p12), cc = pair(c);
    const short2v hi = __builtin_elementwise_min(__builtin_elementwise_max(a, b), __builtin_elementwise_max(r, l));
    const short2v lo = __builtin_elementwise_max(__builtin_elementwise_min(a, b), __builtin_elementwise_min(r, l));
    // sign bit set where tmin - margin < 0, i.e. the margin exceeds tmin
    const uint32_t e = __builtin_bit_cast(uint32_t, (short2v)(tm - (hi - cc))) |
                       __builtin_bit_cast(uint32_t, (short2v)(tm - (cc - lo)));
    res |= ((e >> 15) & 1u) << h;        // byte h
    res |= ((e >> 31) & 1u) << (2 + h);  // byte h + 2
  }
  return res;
}

// FAST-9 score (Sec. III-D): the largest tau with a 9-arc all brighter than
// I(p)+tau or all darker than I(p)-tau, i.e. (max over polarity and arc of the
// arc's minimum signed difference) - 1. Both polarities ride in the two
// 16-bit halves of one register (differences lie in -255..255): sliding
// minima of width 2, 4, then 9 over the circle, one maximum.
__device__ __forceinline__ int fast_score(const int d[16]) {
  short2v e[16], m2[16], m4[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) e[k] = short2v{(short)d[k], (short)-d[k]};
#pragma unroll
  for (int k = 0; k < 16; ++k) m2[k] = __builtin_elementwise_min(e[k], e[(k + 1) & 15]);
#pragma unroll
  for (int k = 0; k < 16; ++k) m4[k] = __builtin_elementwise_min(m2[k], m2[(k + 2) & 15]);
  short2v best = __builtin_elementwise_min(__builtin_elementwise_min(m4[0], m4[4]), e[8]);
#pragma unroll
  for (int k = 1; k < 16; ++k)
    best = __builtin_elementwise_max(
        best, __builtin_elementwise_min(__builtin_elementwise_min(m4[k], m4[(k + 4) & 15]), e[(k + 8) & 15]));
  return max(max((int)best.x, (int)best.y) - 1, -1);
}

typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t* s_v32(uint16_t* p) { return reinterpret_cast<uint32_t*>(p); }

// eq. (2) for two adjacent outputs: with input bytes x0..x6 (x_k = byte k of
// a, then b), out = (x0 + 4 x1 + 6 x2 + 4 x3 + x4, x2 + 4 x3 + 6 x4 + 4 x5 + x6)
// in the low and high 16-bit halves (each at most 16 * 255).
__device__ __forceinline__ uint32_t pyr_h_pair(uint32_t a, uint32_t b) {
  // v_perm_b32 selectors over (b:a): bytes 0..3 of a are 0..3, of b 4..7; 0x0C gives zero
  const ushort2v p0 = __builtin_bit_cast(ushort2v, __builtin_amdgcn_perm(b, a, 0x0C020C00u));  // x0, x2
  const ushort2v p1 = __builtin_bit_cast(ushort2v, __builtin_amdgcn_perm(b, a, 0x0C030C01u));  // x1, x3
  const ushort2v p2 = __builtin_bit_cast(ushort2v, __builtin_amdgcn_perm(b, a, 0x0C040C02u));  // x2, x4
  const ushort2v p3 = __builtin_bit_cast(ushort2v, __builtin_amdgcn_perm(b, a, 0x0C050C03u));  // x3, x5
  const ushort2v p4 = __builtin_bit_cast(ushort2v, __builtin_amdgcn_perm(b, a, 0x0C060C04u));  // x4, x6
  const ushort2v four = {4, 4}, six = {6, 6};
  const ushort2v s = (p0 + p4) + four * (p1 + p3) + six * p2;
  return __builtin_bit_cast(uint32_t, s);
}

// eq. (3) for two adjacent columns: five rows of packed horizontal sums,
// (r0 + 4 r1 + 6 r2 + 4 r3 + r4 + 128) >> 8 per half (at most 16 * 4080 + 128,
// which fits 16 bits), returned as two bytes in the low 16 bits.
__device__ __forceinline__ uint32_t pyr_v_pair(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t r4) {
  const ushort2v v0 = __builtin_bit_cast(ushort2v, r0), v1 = __builtin_bit_cast(ushort2v, r1);
  const ushort2v v2 = __builtin_bit_cast(ushort2v, r2), v3 = __builtin_bit_cast(ushort2v, r3);
  const ushort2v v4 = __builtin_bit_cast(ushort2v, r4);
  const ushort2v four = {4, 4}, six = {6, 6}, half = {128, 128}, eight = {8, 8};
  const ushort2v s = ((v0 + v4) + four * (v1 + v3) + six * v2 + half) >> eight;
  const uint32_t w = __builtin_bit_cast(uint32_t, s);
  return (w & 0xFFu) | ((w >> 8) & 0xFF00u);
}

template <int L, int T>
__global__ __launch_bounds__(T == 64 ? 1024 : 256) void k_pyr_detect(const CamDesc* __restrict__ cams,
                                                                      const FrameTable* __restrict__ frame,
                                                                      FrameTable* __restrict__ dframe,
                                                                      int copy_words, int cam_begin, int cam_end,
                                                                      int tile_base, int tmin, int margin) {
  using G = PyrGeom<L, T>;
  static_assert(G::threads == (T == 64 ? 1024 : 256), "launch bounds");
  constexpr int kTile = T;
  constexpr int kPyrThreads = G::threads;
  constexpr int kScoreEdge = G::score_edge;
  __shared__ __align__(16) uint8_t s_l0[G::sh0 * G::sw0];
  __shared__ __align__(4) uint8_t s_score[G::score_bytes];
  __shared__ uint16_t s_cand[kScoreEdge * kScoreEdge];  // pixels past the early rejection
  __shared__ int s_ncand;
  __shared__ __align__(16) uint16_t s_v[G::vbytes];
  __shared__ __align__(16) uint8_t s_lv[2][G::lvl_bytes];

  // `frame` is the frame's table in mapped pinned host memory; the first
  // workgroup copies it to the device table that the later kernels of the
  // frame read (no separate copy call on the host)
  if (blockIdx.x == 0) {
    const uint32_t* fs = reinterpret_cast<const uint32_t*>(frame);
    uint32_t* fd = reinterpret_cast<uint32_t*>(dframe);
    for (int i = (int)threadIdx.x; i < copy_words; i += kPyrThreads) fd[i] = fs[i];
  }
  const int gtile = tile_base + xcd_tile<G::xcd_run>((int)blockIdx.x, (int)gridDim.x);
  int c = cam_begin;
  while (c + 1 < cam_end && cams[c + 1].tile_begin <= gtile) ++c;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active) return;
  const int t = gtile - cd.tile_begin;
  const int x0 = (t % cd.tiles_x) * kTile, y0 = (t / cd.tiles_x) * kTile;
  const int W = cd.w, H = cd.h, par = fc.pyr;
  const int tid = threadIdx.x;

  // ---- stage level 0 (tile + apron) -------------------------------------
  const int ox0 = x0 - G::a0x, oy0 = y0 - G::a0;
  const uint8_t* src = fc.src;
  const int sp = fc.src_pitch;
  const bool aligned = ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)sp) & 3) == 0;
  constexpr int qrow = G::sw0 / 4;
  if (aligned && ox0 >= 0 && oy0 >= 0 && ox0 + G::sw0 <= W && oy0 + G::sh0 <= H) {
    // the whole staged region inside the image (the workgroup's choice): plain dword copies
    for (int i = tid; i < G::sh0 * qrow; i += kPyrThreads) {
      const int r = i / qrow, q = i - r * qrow;
      *reinterpret_cast<uint32_t*>(&s_l0[r * G::sw0 + 4 * q]) =
          *reinterpret_cast<const uint32_t*>(src + (size_t)(oy0 + r) * sp + ox0 + 4 * q);
    }
  } else
  for (int i = tid; i < G::sh0 * qrow; i += kPyrThreads) {
    const int r = i / qrow, q = i - r * qrow;
    const int y = oy0 + r, x = ox0 + 4 * q;
    uint32_t v = 0;
    if (y >= 0 && y < H) {
      const uint8_t* row = src + (size_t)y * sp;
      if (aligned && x >= 0 && x + 3 < W) {
        v = *reinterpret_cast<const uint32_t*>(row + x);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (x + k >= 0 && x + k < W) v |= (uint32_t)row[x + k] << (8 * k);
      }
    }
    *reinterpret_cast<uint32_t*>(&s_l0[r * G::sw0 + 4 * q]) = v;
  }
  if (tid == 0) s_ncand = 0;
  __syncthreads();

  // ---- copy level 0 into the own pyramid when it came from outside --------
  if (fc.copy_l0) {
    uint8_t* dst = cd.lvl[par][0];
    const int dp = cd.pitch[0];
    for (int i = tid; i < kTile * (kTile / 4); i += kPyrThreads) {
      const int r = i / (kTile / 4), q = i - r * (kTile / 4);
      const int y = y0 + r, x = x0 + 4 * q;
      if (y >= H || x >= W) continue;
      const uint8_t* s = &s_l0[(y - oy0) * G::sw0 + (x - ox0)];
      if (x + 3 < W) {
        *reinterpret_cast<uint32_t*>(dst + (size_t)y * dp + x) = *reinterpret_cast<const uint32_t*>(s);
      } else {
        for (int k = 0; x + k < W; ++k) dst[(size_t)y * dp + x + k] = s[k];
      }
    }
  }

  // ---- FAST-9 + strict NMS + per-cell key ---------------------------------
  // Scores of the tile and its one-pixel ring (0: below the last threshold).
  // The early rejection runs over every pixel and appends the survivors (about
  // a quarter of a textured image) to a list; the full score then runs over
  // the list, so a wave scores 64 survivors at a time instead of running the
  // score for every wave that holds one.
  if (cd.detect) {
    const int lane = tid & 63;
    for (int i = tid; i < G::score_bytes / 4; i += kPyrThreads) reinterpret_cast<uint32_t*>(s_score)[i] = 0u;
    // four pixels per thread: the score-region row cy, columns 4g-3 .. 4g
    constexpr int kGroups = G::fast_groups, kItems = kScoreEdge * kGroups;
    for (int i0 = 0; i0 < kItems; i0 += kPyrThreads) {  // the same trip count for every thread
      const int it = i0 + tid;
      const int cy = it / kGroups, g = it - cy * kGroups;
      const int cx0 = 4 * g - 3;
      const int sy = y0 - 1 + cy, sx0 = x0 - 1 + cx0;
      // bytes k of the group that are score-region pixels inside the margins
      const int klo = max(max(0, -cx0), margin - 1 - sx0);
      const int khi = min(min(3, kScoreEdge - 1 - cx0), W - margin - sx0);
      const bool rows_ok = it < kItems && sy >= margin - 1 && sy <= H - margin && klo <= khi;
      uint32_t m = 0;
      if (rows_ok) {
        const int lx = 4 * g + G::a0x - 4;
        const uint8_t* row = s_l0 + (cy + G::a0 - 1) * G::sw0;
        const uint32_t up = *reinterpret_cast<const uint32_t*>(row - 3 * G::sw0 + lx);
        const uint32_t dn = *reinterpret_cast<const uint32_t*>(row + 3 * G::sw0 + lx);
        // (at lx = 0 the left dword is not needed: only byte 3 is a pixel then)
        const uint32_t w0 = *reinterpret_cast<const uint32_t*>(row + max(lx - 4, 0));
        const uint32_t c = *reinterpret_cast<const uint32_t*>(row + lx);
        const uint32_t w2 = *reinterpret_cast<const uint32_t*>(row + lx + 4);
        const uint32_t lt = __builtin_amdgcn_alignbyte(c, w0, 1), rt = __builtin_amdgcn_alignbyte(w2, c, 3);
        m = fast_may_pass4(up, rt, dn, lt, c, tmin) & ((2u << khi) - (1u << klo));
      }
      // the wave's candidates go to consecutive slots: a scan of the counts,
      // one LDS atomic per wave
      const int n = __popc(m);
      const int incl = wave_incl_scan(n);
      const int tot = __builtin_amdgcn_readlane(incl, 63);
      if (tot) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_ncand, tot);
        int at = __builtin_amdgcn_readlane(base, 0) + incl - n;
        const int i_row = cy * kScoreEdge + cx0;
        while (m) {
          const int k = __ffs(m) - 1;
          m &= m - 1;
          s_cand[at++] = (uint16_t)(i_row + k);
        }
      }
    }
    __syncthreads();
    const int ncand = s_ncand;
    for (int j = tid; j < ncand; j += kPyrThreads) {
      const int i = s_cand[j];
      const int sy = y0 - 1 + i / kScoreEdge, sx = x0 - 1 + i % kScoreEdge;
      int d[16];
      ring_diffs(s_l0, (sy - oy0) * G::sw0 + (sx - ox0), G::sw0, d);
      const int score = fast_score(d);
      s_score[i] = (uint8_t)(score >= tmin ? score + 1 : 0);
    }
    __syncthreads();
    // strict 3x3 maxima: only listed pixels can hold a nonzero score
    uint32_t* keys = cd.keys[par];
    for (int j = tid; j < ncand; j += kPyrThreads) {
      const int i = s_cand[j];
      const int ly = i / kScoreEdge - 1, lx = i % kScoreEdge - 1;
      const int x = x0 + lx, y = y0 + ly;
      // branch-free test: tile pixels inside the margins (the ring around the
      // tile and margin pixels read an interior slot instead, and fail)
      const bool inside = (unsigned)lx < (unsigned)kTile && (unsigned)ly < (unsigned)kTile && x >= margin &&
                          x <= W - 1 - margin && y >= margin && y <= H - 1 - margin;
      const uint8_t* sc = &s_score[inside ? i : kScoreEdge + 1];
      const int s = sc[0];
      const bool peak = inside & (s != 0) & (s > sc[-kScoreEdge - 1]) & (s > sc[-kScoreEdge]) &
                        (s > sc[-kScoreEdge + 1]) & (s > sc[-1]) & (s > sc[1]) & (s > sc[kScoreEdge - 1]) &
                        (s > sc[kScoreEdge]) & (s > sc[kScoreEdge + 1]);
      // the caller's detection mask drops a corner after the maximum test, so
      // a masked maximum still suppresses its neighbours
      if (peak && (!cd.has_mask || cd.mask[y * W + x] == 0)) {
        const uint32_t key = ((uint32_t)(s - 1) << 24) | (0xFFFFFFu - (uint32_t)(y * W + x));
        const int cell = (y / cd.cell) * cd.ncx + x / cd.cell;
        if (cd.kcell == 1) {
          atomicMax(&keys[cell], key);
        } else {
          // k > 1: the cell's k slots keep its best keys in descending order.
          // Each slot keeps the larger of its value and the incoming key and
          // passes the smaller one on, so slot values plus keys in flight
          // always form the same multiset; once every insert has finished,
          // slot r holds the (r+1)-th largest key (0 = none).
          uint32_t* slot = keys + cell * cd.kcell;
          uint32_t v = key;
          for (int r = 0; r < cd.kcell && v != 0u; ++r) v = min(v, atomicMax(&slot[r], v));
        }
      }
    }
  }

  // ---- coarser levels from LDS (eqs. 2-3) ---------------------------------
  if constexpr (L > 1) {
    const uint8_t* cur = s_l0;
    int cur_ox = ox0, cur_oy = oy0, cur_p = G::sw0;
#pragma unroll
    for (int l = 0; l < L - 1; ++l) {
      const int Wc = W >> l, Hc = H >> l, Wn = W >> (l + 1), Hn = H >> (l + 1);
      const int S = G::region(l + 1);
      const int o_x = (x0 >> (l + 1)) - G::apron(l + 1), o_y = (y0 >> (l + 1)) - G::apron(l + 1);
      const int X0 = max(0, o_x), X1 = min(Wn - 1, o_x + S - 1);
      const int Y0 = max(0, o_y), Y1 = min(Hn - 1, o_y + S - 1);
      const int vy0 = max(0, 2 * o_y - 2), vy1 = min(Hc - 1, 2 * (o_y + S - 1) + 2);
      // passes run over the full region width S (a compile-time constant, so
      // the index split is a multiply-shift) and skip columns outside the image
      // block-uniform: a level with nothing inside the image ends the tile
      if (X0 > X1 || Y0 > Y1) break;
      // a region wholly inside the image with every filter tap inside level l
      // (no clamping) runs two outputs per thread in packed 16-bit halves
      const bool paired = G::region(l) % 4 == 0 && S % 4 == 0 && (kTile >> (l + 1)) % 2 == 0 && X0 == o_x &&
                          X1 == o_x + S - 1 && 2 * o_x - 2 >= 0 &&
                          2 * X1 + 2 <= Wc - 1 && 2 * Y0 - 2 >= 0 && 2 * Y1 + 2 <= Hc - 1;
      if (paired) {
        const int shift = l == 0 ? G::h_shift0 : 0;
        const int npair = S / 2;
        // eq. (2): outputs X, X+1 from input bytes 2X-2 .. 2X+4
        const int nv = (vy1 - vy0 + 1) * npair;
        for (int i = tid; i < nv; i += kPyrThreads) {
          const int r = i / npair, q = i - r * npair;
          const uint32_t* w = reinterpret_cast<const uint32_t*>(cur + (vy0 + r - cur_oy) * cur_p) + q;
          const uint32_t d0 = w[0], d1 = w[1], d2 = shift != 0 ? w[2] : 0u;
          const uint32_t a = __builtin_amdgcn_alignbyte(d1, d0, shift);  // bytes 0..3 of the window
          const uint32_t b = __builtin_amdgcn_alignbyte(d2, d1, shift);  // bytes 4..7
          s_v32(s_v)[r * npair + q] = pyr_h_pair(a, b);
        }
        __syncthreads();
        // eq. (3): +128 then >> 8, two columns per thread
        uint8_t* nxt = s_lv[l & 1];
        uint8_t* gdst = cd.lvl[par][l + 1];
        const int gp = cd.pitch[l + 1];
        const int tx0 = x0 >> (l + 1), ty0 = y0 >> (l + 1), te = kTile >> (l + 1);
        const int nn = (Y1 - Y0 + 1) * npair;
        for (int i = tid; i < nn; i += kPyrThreads) {
          const int Y = Y0 + i / npair, q = i % npair;
          const uint32_t* col = s_v32(s_v) + (2 * Y - 2 - vy0) * npair + q;
          const uint32_t v2 = pyr_v_pair(col[0], col[npair], col[2 * npair], col[3 * npair], col[4 * npair]);
          const int X = o_x + 2 * q;
          *reinterpret_cast<uint16_t*>(&nxt[(Y - o_y) * S + 2 * q]) = (uint16_t)v2;
          if (X >= tx0 && X < tx0 + te && Y >= ty0 && Y < ty0 + te)
            *reinterpret_cast<uint16_t*>(&gdst[(size_t)Y * gp + X]) = (uint16_t)v2;
        }
        __syncthreads();
        cur = nxt;
        cur_ox = o_x;
        cur_oy = o_y;
        cur_p = S;
      } else {
        // eq. (2): horizontal pass over level-l rows vy0..vy1
        const int nv = (vy1 - vy0 + 1) * S;
        for (int i = tid; i < nv; i += kPyrThreads) {
          const int r = i / S, X = o_x + i % S;
          if (X < X0 || X > X1) continue;
          const uint8_t* row = cur + (vy0 + r - cur_oy) * cur_p - cur_ox;
          const int xa = 2 * X;
          const uint32_t v = row[clampi(xa - 2, 0, Wc - 1)] + 4u * row[clampi(xa - 1, 0, Wc - 1)] +
                             6u * row[xa] + 4u * row[clampi(xa + 1, 0, Wc - 1)] + row[clampi(xa + 2, 0, Wc - 1)];
          s_v[r * S + (X - o_x)] = (uint16_t)v;
        }
        __syncthreads();
        // eq. (3): vertical pass, +128 then >> 8
        uint8_t* nxt = s_lv[l & 1];
        uint8_t* gdst = cd.lvl[par][l + 1];
        const int gp = cd.pitch[l + 1];
        const int tx0 = x0 >> (l + 1), ty0 = y0 >> (l + 1), te = kTile >> (l + 1);
        const int nn = (Y1 - Y0 + 1) * S;
        for (int i = tid; i < nn; i += kPyrThreads) {
          const int Y = Y0 + i / S, X = o_x + i % S;
          if (X < X0 || X > X1) continue;
          const uint16_t* col = s_v + (X - o_x);
          const int ya = 2 * Y;
          const uint32_t s = col[(clampi(ya - 2, 0, Hc - 1) - vy0) * S] + 4u * col[(clampi(ya - 1, 0, Hc - 1) - vy0) * S] +
                             6u * col[(ya - vy0) * S] + 4u * col[(clampi(ya + 1, 0, Hc - 1) - vy0) * S] +
                             col[(clampi(ya + 2, 0, Hc - 1) - vy0) * S];
          const uint8_t val = (uint8_t)((s + 128u) >> 8);
          nxt[(Y - o_y) * S + (X - o_x)] = val;
          if (X >= tx0 && X < tx0 + te && Y >= ty0 && Y < ty0 + te) gdst[(size_t)Y * gp + X] = val;
        }
        __syncthreads();
        cur = nxt;
        cur_ox = o_x;
        cur_oy = o_y;
        cur_p = S;
      }
    }
  }
}

template <int L, int T>
hipError_t launch_LT(const CamDesc* cams, const FrameTable* frame, FrameTable* dframe, int copy_words, int cam_begin,
                     int cam_end, int tile_base, int n_tiles, int tmin, int margin, hipStream_t s) {
  launch_kernel(k_pyr_detect<L, T>, dim3(n_tiles), dim3(PyrGeom<L, T>::threads), 0, s, cams, frame, dframe, copy_words,
                cam_begin, cam_end, tile_base, tmin, margin);
  return hipGetLastError();
}

template <int T>
size_t lds_bytes_T(int levels) {
  hipFuncAttributes a{};
  hipError_t e = hipErrorInvalidValue;
  switch (levels) {
    case 1: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<1, T>)); break;
    case 2: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<2, T>)); break;
    case 3: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<3, T>)); break;
    case 4: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<4, T>)); break;
    case 5: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<5, T>)); break;
    case 6: e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_pyr_detect<6, T>)); break;
    default: break;
  }
  return e == hipSuccess ? a.sharedSizeBytes : 0;
}

template <int T>
hipError_t launch_T(const CamDesc* d_cams, const FrameTable* h_frame, FrameTable* d_frame, int copy_words, int cam_begin,
                    int cam_end, int tile_base, int n_tiles, int levels, int tmin, int margin, hipStream_t s) {
  switch (levels) {
    case 1: return launch_LT<1, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    case 2: return launch_LT<2, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    case 3: return launch_LT<3, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    case 4: return launch_LT<4, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    case 5: return launch_LT<5, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    case 6: return launch_LT<6, T>(d_cams, h_frame, d_frame, copy_words, cam_begin, cam_end, tile_base, n_tiles, tmin,
                                       margin, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Static LDS bytes of the pyramid/detector kernel for `levels` and tile edge
// `tile` (0 if unknown).
size_t pyr_detect_lds_bytes(int levels, int tile) {
  return tile == 32 ? lds_bytes_T<32>(levels) : tile == 64 ? lds_bytes_T<64>(levels) : 0;
}

hipError_t launch_pyr_detect_range(const CamDesc* d_cams, const FrameTable* h_frame, FrameTable* d_frame,
                                   int copy_bytes, int cam_begin, int cam_end, int tile_base, int n_tiles, int levels,
                                   int tile, int tmin, int margin, hipStream_t s) {
  if (n_tiles <= 0 || copy_bytes % 4) return hipErrorInvalidValue;
  const int w = copy_bytes / 4;
  if (tile == 32)
    return launch_T<32>(d_cams, h_frame, d_frame, w, cam_begin, cam_end, tile_base, n_tiles, levels, tmin, margin, s);
  if (tile == 64)
    return launch_T<64>(d_cams, h_frame, d_frame, w, cam_begin, cam_end, tile_base, n_tiles, levels, tmin, margin, s);
  return hipErrorInvalidValue;
}

}  // namespace vio
