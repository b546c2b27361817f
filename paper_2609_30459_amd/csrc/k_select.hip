// Keypoint bookkeeping after tracking (Sec. III-B/III-D): cell mask, global
// cap, new identifiers, stable compaction of the surviving tracks, acceptance
// of stereo matches and the output records TR_t / DET_t, written straight
// into mapped pinned host memory (the host reads them after the frame's wait,
// with no copy).
//
// One 1024-thread workgroup per stream; camera groups (mono camera or stereo
// pair) are handled in order so identifiers are assigned in (group, cell)
// order. Every ordering decision is a prefix count over flags (wave ballots
// plus a scan of the 16 wave totals), so the result does not depend on thread
// timing.
//
// Rules (all on integers):
//  * a cell is masked when it holds at least k surviving tracks of the camera;
//  * the candidates are the (up to k) winners of the unmasked cells, in key
//    slots cell * k + rank; the best (score desc, cell asc, rank asc) up to
//    cap - live are kept, found with a 256-bin score histogram instead of a
//    sort (equal scores are taken in slot order);
//  * the kept ones get consecutive identifiers in slot (cell, rank) order;
//  * a stereo match is accepted while the right camera has room.
//
// Phases: kSelectAll reads the speculative stereo match of every selected
// winner (indexed by key slot). With deferred stereo matching the work splits in
// two launches around the stereo tracking launch: kSelectLeft does
// everything except the right cameras' matches and leaves the new detections'
// place in the left state in sel_base / n_sel; kSelectRight accepts the
// matches (indexed by selection rank) into the right cameras.
#include "fe_common.h"
#include "wave_ops.h"

namespace vio {

constexpr int kMaxCells = 8192;

namespace {

constexpr int kWaves = kSelectThreads / 64;

struct ScanScratch {
  int wave_tot[2][kWaves];
};

// A thread's handle on the block's scan scratch. Every thread makes the same
// sequence of scan calls, so `tog` agrees across the block.
struct Scan {
  ScanScratch* sh;
  int tog;
};

// Exclusive prefix count of `flag` over the block's threads in thread order;
// returns the thread's offset and sets `total`. All threads must call it.
// One barrier per call: the wave totals alternate between two buffers, and a
// buffer is rewritten two calls later, which a thread reaches only after the
// next call's barrier, i.e. after every thread has read this call's totals.
// Two flags with one barrier: the prefix count of `flag` and both totals (a
// wave's two counts share one word).
__device__ __forceinline__ int block_scan_flag2(bool flag, bool flag2, Scan& sc, int& total, int& total2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag), m2 = __ballot(flag2);
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  int* tot = sc.sh->wave_tot[sc.tog];
  sc.tog ^= 1;
  if (lane == 0) tot[wave] = __popcll(m) | (__popcll(m2) << 16);
  __syncthreads();
  int off = 0, all = 0, all2 = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int t = tot[w];
    off += w < wave ? (t & 0xFFFF) : 0;
    all += t & 0xFFFF;
    all2 += t >> 16;
  }
  total = all;
  total2 = all2;
  return off + below;
}

__device__ __forceinline__ int block_scan_flag(bool flag, Scan& sc, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  int* tot = sc.sh->wave_tot[sc.tog];
  sc.tog ^= 1;
  if (lane == 0) tot[wave] = __popcll(m);
  __syncthreads();
  int off = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int t = tot[w];
    off += w < wave ? t : 0;
    all += t;
  }
  total = all;
  return off + below;
}



__device__ __forceinline__ vio_track make_rec(int64_t id, int cam, int status, float x, float y, float th, float fb,
                                              float res, int age, int score) {
  vio_track t;
  t.id = id;
  t.x = x;
  t.y = y;
  t.theta = th;
  t.fb_err = fb;
  t.resid_rms = res;
  t.age = age;
  t.camera = (int16_t)cam;
  t.status = (int16_t)status;
  t.score = score;
  return t;
}

__device__ __forceinline__ Kp make_kp(int64_t id, float x, float y, float px, float py, int age) {
  Kp k;
  k.id = id;
  k.x = x;
  k.y = y;
  k.px = px;
  k.py = py;
  k.age = age;
  k.reserved = 0;
  return k;
}

// A live keypoint's id and position, kept in LDS for the neighbour stereo
// start's pair table while the selection writes the state.
struct PairRow {
  int64_t id;
  float x, y;
};
constexpr int kPairLds = 1024;  // rows per camera kept in LDS (cameras of larger caps read global memory)

// Carries camera c's previous keypoints into its current state: the survivors
// of temporal tracking (all of them when there was no previous frame) in their
// old order, with their records. Adds the survivors to `occ` when given, and
// their ids and positions to `tab` when given. Returns the survivor count;
// *n_rec receives the number of records written.
__device__ int carry_survivors(const CamDesc& cd, const FrameCam& fc, int n_prev, unsigned* occ, Scan& sc,
                               int* n_rec, bool count_fallback, PairRow* tab = nullptr,
                               int64_t* tab_ids = nullptr) {
  const int P = fc.parity, Q = P ^ 1;
  int base = 0, n_fb = 0;
  for (int j0 = 0; j0 < n_prev; j0 += kSelectThreads) {
    const int j = j0 + (int)threadIdx.x;
    bool alive = false;
    Kp kp{};
    TrackRes r{};
    if (j < n_prev) {
      kp = cd.state[Q][j];
      if (fc.has_prev) {
        // a short attempt that was not kept: its fallback, computed beside it
        // (both results loaded at once, so the choice costs no second round
        // trip; the fallback slot of a kept track is not used)
        r = cd.res[j];
        if (cd.res_fb) {
          const TrackRes rf = cd.res_fb[j];
          if (r.pad[0] != 0) r = rf;
        }
        alive = r.status == VIO_TRACKED;
      } else {
        r.x = kp.x;
        r.y = kp.y;
        alive = true;
      }
    }
    int total, fb_tot;
    const int pos = base + (count_fallback ? block_scan_flag2(alive, j < n_prev && fc.has_prev && r.pad[0] != 0, sc,
                                                              total, fb_tot)
                                           : block_scan_flag(alive, sc, total));
    if (count_fallback) n_fb += fb_tot;
    if (j < n_prev) {
      if (alive) {
        if (occ) {
          const int cx = (int)floorf(r.x / (float)cd.cell), cy = (int)floorf(r.y / (float)cd.cell);
          if (cx >= 0 && cx < cd.ncx && cy >= 0 && cy < cd.ncy) atomicAdd(&occ[cy * cd.ncx + cx], 1u);
        }
        cd.state[P][pos] = fc.has_prev ? make_kp(kp.id, r.x, r.y, kp.x, kp.y, kp.age + 1) : kp;
        if (tab) tab[pos] = PairRow{kp.id, fc.has_prev ? r.x : kp.x, fc.has_prev ? r.y : kp.y};
        if (tab_ids) tab_ids[pos] = kp.id;
      }
      if (fc.has_prev)
        cd.rec[fc.rec_slot][j] = make_rec(kp.id, cd.local, r.status, r.x, r.y, r.theta, r.fb, r.resid,
                             alive ? kp.age + 1 : kp.age, -1);
    }
    base += total;
  }
  *n_rec = fc.has_prev ? n_prev : 0;
  if (threadIdx.x == 0) {
    int32_t* st = cd.stats_out[fc.rec_slot];
    st[kStatFallback] = n_fb;
    st[kStatTracked] = fc.has_prev ? base : 0;
    st[kStatLost] = fc.has_prev ? n_prev - base : 0;
    st[kStatDetected] = 0;
    st[kStatMatched] = 0;
  }
  return base;
}

// Appends the accepted stereo matches of the n_new detections of left camera
// L (ids from L's new keypoints state[P][sel_base + i]) to right camera R,
// after its n_surv_r survivors and n_rec_r temporal records. sres(i): the
// match of detection i.
template <class SresOf>
__device__ int accept_matches(const CamDesc& L, int P, int sel_base, const CamDesc& R, const FrameCam& fr,
                              int rc, int n_new, int n_surv_r, int n_rec_r, SresOf sres, Counters* cnt,
                              Scan& sc, PairRow* tab = nullptr) {
  const int PR = fr.parity;
  int m_base = 0;
  for (int i0 = 0; i0 < n_new; i0 += kSelectThreads) {
    const int i = i0 + (int)threadIdx.x;
    const bool valid = i < n_new;
    TrackRes sr{};
    int64_t id = 0;
    if (valid) {
      sr = sres(i);
      id = L.state[P][sel_base + i].id;
    }
    const bool matched = valid && sr.status == VIO_TRACKED;
    int m_tot;
    const int mrank = m_base + block_scan_flag(matched, sc, m_tot);
    if (valid) {
      const bool accepted = matched && n_surv_r + mrank < R.cap;
      const int st = matched ? (accepted ? VIO_MATCHED : VIO_LOST_CAP) : sr.status;
      R.rec[fr.rec_slot][n_rec_r + i] = make_rec(id, R.local, st, sr.x, sr.y, sr.theta, sr.fb, sr.resid, 0, -1);
      if (accepted) {
        R.state[PR][n_surv_r + mrank] = make_kp(id, sr.x, sr.y, sr.x, sr.y, 0);
        if (tab) tab[n_surv_r + mrank] = PairRow{id, sr.x, sr.y};
      }
    }
    m_base += m_tot;
  }
  const int accepted = min(m_base, max(0, R.cap - n_surv_r));
  if (threadIdx.x == 0) {
    cnt->n_live[PR][rc] = n_surv_r + accepted;
    cnt->rec_count[rc] = n_rec_r + n_new;
    *R.rec_count_out[fr.rec_slot] = n_rec_r + n_new;
    R.stats_out[fr.rec_slot][kStatMatched] = accepted;
  }
  return n_surv_r + accepted;
}

// The neighbour stereo start's table of target camera R (parity PR): its
// n_right keypoints, in id order, that also live among detecting camera L's
// n_left keypoints (parity P; both states are sorted by id), as L's position
// and the offset from L to R. The next frame's stereo matches into R read it.
// tl / tr: both cameras' ids and positions as the selection wrote them to
// LDS (when they fit; tl_ids: the left ids again, contiguous, for the
// search), else the states in memory, with the left ids staged in s_ids (LDS
// room for kPairIdsLds ids) when they fit there.
constexpr int kPairIdsLds = kMaxCells / 2;  // int64 ids in the occupancy array's bytes

__device__ void build_pairs(const CamDesc& L, int P, int n_left, const CamDesc& R, int PR, int rc, int n_right,
                            Counters* cnt, Scan& sc, const PairRow* tl, const int64_t* tl_ids, const PairRow* tr,
                            int64_t* s_ids) {
  const bool staged = !tl && n_left <= kPairIdsLds;
  if (staged) {
    __syncthreads();  // the LDS array's previous use is over
    for (int k = (int)threadIdx.x; k < n_left; k += kSelectThreads) s_ids[k] = L.state[P][k].id;
    __syncthreads();
  }
  int base = 0;
  for (int i0 = 0; i0 < n_right; i0 += kSelectThreads) {
    const int i = i0 + (int)threadIdx.x;
    bool found = false;
    float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n_right) {
      int64_t qid;
      float qx, qy;
      if (tr) {
        const PairRow q = tr[i];
        qid = q.id;
        qx = q.x;
        qy = q.y;
      } else {
        const Kp q = R.state[PR][i];
        qid = q.id;
        qx = q.x;
        qy = q.y;
      }
      int at = -1;
      if (tl_ids) {
        // lower bound over the contiguous LDS ids, branch-free: every lane
        // takes the same floor(log2(n_left)) + 1 steps of halving size
        if (n_left > 0) {
          int pos = 0;  // ids below qid so far
          for (int step = 1 << (31 - __clz(n_left)); step > 0; step >>= 1) {
            const int probe = pos + step;
            const int64_t v = tl_ids[min(probe, n_left) - 1];
            pos = probe <= n_left && v < qid ? probe : pos;
          }
          at = pos < n_left && tl_ids[pos] == qid ? pos : -1;
        }
      } else {
        int lo = 0, hi = n_left - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int64_t id = staged ? s_ids[mid] : L.state[P][mid].id;
          if (id == qid) {
            at = mid;
            break;
          }
          if (id < qid) lo = mid + 1;
          else hi = mid - 1;
        }
      }
      if (at >= 0) {
        float lx, ly;
        if (tl) {
          lx = tl[at].x;
          ly = tl[at].y;
        } else {
          const Kp l = L.state[P][at];
          lx = l.x;
          ly = l.y;
        }
        e = make_float4(lx, ly, qx - lx, qy - ly);
        found = true;
      }
    }
    int total;
    const int pos = base + block_scan_flag(found, sc, total);
    if (found) R.pairs[PR][pos] = e;
    base += total;
  }
  if (threadIdx.x == 0) cnt->n_pairs[PR][rc] = base;
}

__global__ __launch_bounds__(kSelectThreads) void k_select(const CamDesc* __restrict__ cams,
                                                          const FrameTable* __restrict__ frame, Counters* cnt,
                                                          const int* __restrict__ stream_cams, int phase,
                                                          Tuning tune) {
  __shared__ ScanScratch s_scan;
  __shared__ int s_hsum[4];
  Scan sc{&s_scan, 0};
  __shared__ __align__(8) unsigned s_occ[kMaxCells];  // cell occupancy; later the pair search's left ids
  __shared__ uint16_t s_sel[kMaxCells];  // key slot of selection rank i (rank < cap <= kMaxCells, slot < 2^16)
  __shared__ int s_hist[256];
  __shared__ int s_thr[2];
  // the detecting and the target camera's rows for the neighbour stereo start's pair table
  __shared__ PairRow s_pl[kPairLds], s_pr[kPairLds];
  __shared__ int64_t s_plid[kPairLds];  // s_pl's ids, contiguous for the pair search
  const int s = blockIdx.x;
  const int cam0 = stream_cams[2 * s], ncam = stream_cams[2 * s + 1];
  if (!frame->cam[cam0].active) return;
  // camera groups: a detecting camera followed by the n_targets cameras that
  // receive its matches (mono: none, stereo pair: one, star rig: three)
  if (phase == kSelectRight) {
    for (int g = 0; g < ncam; g += 1 + cams[cam0 + g].n_targets) {
      const int lc = cam0 + g;
      const CamDesc& L = cams[lc];
      const int P = frame->cam[lc].parity;
      for (int t = 0; t < L.n_targets; ++t) {
        const int rc = lc + 1 + t;
        const FrameCam& fr = frame->cam[rc];
        const int PR = fr.parity;
        const int n_rec_r = fr.has_prev ? cnt->n_live[PR ^ 1][rc] : 0;
        const TrackRes* sr = L.sres + (size_t)t * L.nslots;
        const int n_r = accept_matches(L, P, cnt->sel_base[lc], cams[rc], fr, rc, cnt->n_sel[lc],
                                       cnt->n_live[PR][rc], n_rec_r, [&](int i) { return sr[i]; }, cnt, sc);
        __syncthreads();
        if (tune.stereo_nb) {
          build_pairs(L, P, cnt->sel_base[lc] + cnt->n_sel[lc], cams[rc], PR, rc, n_r, cnt, sc, nullptr, nullptr,
                      nullptr, reinterpret_cast<int64_t*>(s_occ));
          __syncthreads();
        }
      }
    }
    return;
  }
  const int stream = cams[cam0].stream;
  const int64_t id0 = cnt->next_id[stream];
  int64_t next_id = id0;
  for (int g = 0; g < ncam; g += 1 + cams[cam0 + g].n_targets) {
    const int lc = cam0 + g;
    const CamDesc& L = cams[lc];
    const FrameCam& fl = frame->cam[lc];
    const int P = fl.parity, Q = P ^ 1;
    const int ncells = L.ncells, kc = L.kcell, nslots = L.nslots;
    for (int i = threadIdx.x; i < ncells; i += kSelectThreads) s_occ[i] = 0;
    for (int i = threadIdx.x; i < 256; i += kSelectThreads) s_hist[i] = 0;
    __syncthreads();

    // ---- left / mono camera: survivors and occupancy ----------------------
    int n_rec = 0;
    const bool count_fb = tune.learned != 0 || tune.plevels > 0;
    // pair rows in LDS (all-in-one selection with the neighbour stereo start)
    const bool pairs_lds = phase == kSelectAll && tune.stereo_nb && L.cap <= kPairLds;
    const int n_surv = carry_survivors(L, fl, cnt->n_live[Q][lc], s_occ, sc, &n_rec, count_fb,
                                       pairs_lds ? s_pl : nullptr, pairs_lds ? s_plid : nullptr);
    __syncthreads();

    // ---- candidates of unmasked cells, score histogram --------------------
    const uint32_t* keys = L.keys[fl.pyr];
    for (int i = threadIdx.x; i < nslots; i += kSelectThreads) {
      const uint32_t key = keys[i];
      if (key && (int)s_occ[i / kc] < kc) atomicAdd(&s_hist[key >> 24], 1);
    }
    __syncthreads();
    // Score threshold of the best `room` candidates: thread t < 256 holds bin
    // v = 255 - t, so a scan in thread order gives cum(v) = #candidates
    // scoring >= v. With more candidates than room, thr is the bin where cum
    // first reaches room and rem the number taken from it; thr = 256 takes
    // none (no room), thr = -1 takes all.
    {
      const int room = max(0, L.cap - n_surv);
      int hv = 0, incl = 0;
      if (threadIdx.x < 256) {
        hv = s_hist[255 - threadIdx.x];
        incl = wave_incl_scan(hv);
        if ((threadIdx.x & 63) == 63) s_hsum[threadIdx.x >> 6] = incl;
      }
      __syncthreads();
      if (threadIdx.x < 256) {
        const int w = threadIdx.x >> 6;
        int before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int t = s_hsum[k];
          before += k < w ? t : 0;
          total += t;
        }
        const int cum = before + incl;
        if (room > 0 && total > room && cum >= room && cum - hv < room) {
          s_thr[0] = 255 - (int)threadIdx.x;
          s_thr[1] = room - (cum - hv);
        }
        if (threadIdx.x == 0 && (room == 0 || total <= room)) {
          s_thr[0] = room == 0 ? 256 : -1;
          s_thr[1] = 0;
        }
      }
      __syncthreads();
    }
    const int thr = s_thr[0], rem = s_thr[1];

    // ---- selection in slot order, identifiers, DET_t records --------------
    int n_new = 0, eq_base = 0;
    for (int i0 = 0; i0 < nslots; i0 += kSelectThreads) {
      const int slot = i0 + (int)threadIdx.x;
      const uint32_t key = slot < nslots ? keys[slot] : 0u;
      const bool cand = key && (int)s_occ[slot < nslots ? slot / kc : 0] < kc;
      const int score = (int)(key >> 24);
      const bool is_eq = cand && score == thr;
      int eq_tot, sel_tot;
      const int eq_rank = eq_base + block_scan_flag(is_eq, sc, eq_tot);
      const bool sel = cand && (score > thr || (is_eq && eq_rank < rem));
      const int rank = n_new + block_scan_flag(sel, sc, sel_tot);
      if (sel) {
        const int idx = 0xFFFFFF - (int)(key & 0xFFFFFFu);
        const float x = (float)(idx % L.w), y = (float)(idx / L.w);
        const int64_t id = next_id + rank;
        L.state[P][n_surv + rank] = make_kp(id, x, y, x, y, 0);
        if (pairs_lds) {
          s_pl[n_surv + rank] = PairRow{id, x, y};
          s_plid[n_surv + rank] = id;
        }
        L.rec[fl.rec_slot][n_rec + rank] = make_rec(id, L.local, VIO_DETECTED, x, y, 0.f, 0.f, 0.f, 0, score);
        s_sel[rank] = (uint16_t)slot;
      }
      eq_base += eq_tot;
      n_new += sel_tot;
    }
    if (threadIdx.x == 0) {
      cnt->n_live[P][lc] = n_surv + n_new;
      cnt->rec_count[lc] = n_rec + n_new;
      *L.rec_count_out[fl.rec_slot] = n_rec + n_new;
      L.stats_out[fl.rec_slot][kStatDetected] = n_new;
    }
    // the key buffer of the frame kPyrSlots - 1 frames ahead: the frames in
    // between may already run their detectors beside this selection (their
    // buffers were cleared by earlier selections), and that frame cannot be
    // submitted before this one has completed
    uint32_t* next_keys = L.keys[(fl.pyr + kPyrSlots - 1) % kPyrSlots];
    for (int i = threadIdx.x; i < nslots; i += kSelectThreads) next_keys[i] = 0u;
    __syncthreads();

    // ---- target cameras (a pair's right camera, a star's other three):
    //      survivors, then accepted stereo matches
    for (int t = 0; t < L.n_targets; ++t) {
      const int rc = lc + 1 + t;
      const CamDesc& R = cams[rc];
      const FrameCam& fr = frame->cam[rc];
      const int PR = fr.parity;
      int n_rec_r = 0;
      const bool pairs_lds_r = pairs_lds && R.cap <= kPairLds;
      const int n_surv_r = carry_survivors(R, fr, cnt->n_live[PR ^ 1][rc], nullptr, sc, &n_rec_r, count_fb,
                                           pairs_lds_r ? s_pr : nullptr);
      if (phase == kSelectAll) {
        const TrackRes* sr = L.sres + (size_t)t * nslots;
        const int n_r = accept_matches(L, P, n_surv, R, fr, rc, n_new, n_surv_r, n_rec_r,
                                       [&](int i) { return sr[s_sel[i]]; }, cnt, sc, pairs_lds_r ? s_pr : nullptr);
        if (tune.stereo_nb) {
          __syncthreads();
          build_pairs(L, P, n_surv + n_new, R, PR, rc, n_r, cnt, sc, pairs_lds ? s_pl : nullptr,
                      pairs_lds ? s_plid : nullptr, pairs_lds_r ? s_pr : nullptr, reinterpret_cast<int64_t*>(s_occ));
        }
      } else if (threadIdx.x == 0) {
        // the matches come from the stereo tracking launch; kSelectRight appends them
        cnt->sel_base[lc] = n_surv;
        cnt->n_sel[lc] = n_new;
        cnt->n_live[PR][rc] = n_surv_r;
      }
      __syncthreads();
    }
    next_id += n_new;
  }
  if (threadIdx.x == 0) cnt->next_id[stream] = next_id;
}

}  // namespace

hipError_t launch_select(const CamDesc* d_cams, const FrameTable* d_frame, Counters* d_cnt, const int* d_stream_cams,
                         int n_streams_launch, int phase, Tuning tune, hipStream_t s) {
  if (n_streams_launch <= 0) return hipSuccess;
  launch_kernel(k_select, dim3(n_streams_launch), dim3(kSelectThreads), 0, s, d_cams, d_frame, d_cnt,
                d_stream_cams, phase, tune);
  return hipGetLastError();
}

}  // namespace vio
