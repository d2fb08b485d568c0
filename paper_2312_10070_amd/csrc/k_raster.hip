// Per-tile compositing. One 256-thread workgroup per (view, tile) item, one
// pixel per lane: each wave covers an 8x8 pixel block of the tile and each
// 16-lane row of a wave (one DPP row) a 4x4 quadrant of that block. Gaussian
// records of the item's depth-sorted list are staged through LDS in batches
// (one coalesced fetch per record per workgroup). Skipping a record for a
// block or quadrant cannot change the result: outside its support box (taken
// with a small slack) a Gaussian's alpha stays below alpha_min by more than
// FP32 rounding, and the ellipse test keeps a margin too.
//
// Forward: front to back (Eq. 3 colour, Eq. 4 alpha, Eq. 6 depth), batches of
// 448 records (the largest that keeps six workgroups per CU in LDS). Each
// wave tests, 64 records at a time, which records can reach alpha >=
// alpha_min in its block (support box, then an exact ellipse-versus-rectangle
// test) and in which of its quadrants (support box), and appends their LDS
// offsets to one visit list per quadrant. The four rows
// of the wave then walk their own lists side by side, each lane reading its
// row's record from LDS, so a record is visited only by the quadrants it can
// reach; a row whose list has ended reads an all-zero record (alpha = 0). A
// lane stops before the Gaussian that would take its transmittance below
// T_min; a quadrant whose lanes have all stopped gets no further entries, a
// wave leaves the batch as soon as all its lanes have stopped, and the
// workgroup stops fetching batches once all four waves have.
//
// Backward: back to front from each pixel's last composited Gaussian. The
// transmittance in front of Gaussian j is recomputed as T_j = T_{j+1} /
// (1 - alpha_j) instead of being stored; suffix sums of c alpha T and z alpha
// T give the second terms of dC/dalpha and Eq. 8. Per pair, ten partials
// (sums of q (dx, dy, dx^2, dx dy, dy^2) with q = dL/dp / ln 2 for
// alpha = o 2^p, then opacity, colour, direct depth) are summed over pixels
// by DPP / permlane field-splitting reductions. Two walks:
//  - block walk (all ten fields, mapping): batches of 512 records, one visit
//    list per wave (records reaching its 8x8 block), walked one record at a
//    time with the record broadcast from LDS; a wave's sums go out with one
//    10-lane atomic per (Gaussian, wave);
//  - quadrant walk (the six fields of a pose-only backward, tracking):
//    batches of 256 records, one visit list per 4x4 quadrant, the four rows
//    of a wave walking their own lists side by side; a row's sums are added
//    to per-record accumulators in LDS, flushed with one atomic per
//    (Gaussian, tile, field) after each batch.
// A deterministic variant of each stores the wave's (row's) sums per (list
// position, block or quadrant) instead and a second pass adds them per
// Gaussian in a fixed order.
//
// Launch shapes: one workgroup per item (items dealt to XCDs in contiguous
// runs), or a persistent grid whose workgroups pull items from a counter in
// longest-list-first order until the queue is empty (multi-keyframe mapping).
#include "gsr_internal.h"

namespace gsr {

namespace {

// Records staged in LDS per batch (forward, backward block walk, backward
// quadrant walk), capacity of a
// quadrant's visit list, and the LDS slot of an all-zero record (u = v = 0,
// zero conic, o = 0: alpha = 0 at every pixel), which a row reads once its
// list has ended.
constexpr int kFwdBatch = 448;
constexpr int kBwdBatch = 512;
constexpr int kQuadBatch = 256;
constexpr int kListCap = 128;
constexpr int kWavesPerTile = kTileThreads / kWave;
static_assert(kFwdBatch % kWave == 0 && kBwdBatch % kWave == 0 && kQuadBatch % kWave == 0 && kListCap >= kWave,
              "batch / list shape");

struct Block {
  int x0, x1, y0, y1;  // inclusive pixel rectangle of a wave (8x8)
};

struct Pixel {
  int tile, view;
  int px, py;
  int quad;     // 4x4 quadrant of the block (row-major) = DPP row of the lane
  bool inside;
  float fpx, fpy;
  int64_t p;    // pixel index inside the view
  int64_t off;  // view * W * H
  Block blk;
};

// Each wave covers one 8x8 pixel block of the tile (a square block meets fewer
// support boxes than a 16x4 or 32x2 strip), the four blocks row-major in the
// tile; lane row r = lane / 16 covers quadrant r of the block (row-major),
// lanes row-major in the quadrant.
__device__ __forceinline__ Pixel item_pixel(const Raster& Rr, int item) {
  Pixel q;
  q.view = item / Rr.n_tiles;
  q.tile = item - q.view * Rr.n_tiles;
  const int tyi = q.tile / Rr.ntx, txi = q.tile - tyi * Rr.ntx;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int bpr_log2 = Rr.tw_log2 - 3;  // 8x8 blocks per tile row: 1, 2 or 4
  const int bx = w & ((1 << bpr_log2) - 1), by = w >> bpr_log2;
  q.blk.x0 = txi * Rr.tw + 8 * bx;
  q.blk.x1 = q.blk.x0 + 7;
  q.blk.y0 = tyi * Rr.th + 8 * by;
  q.blk.y1 = q.blk.y0 + 7;
  q.quad = l >> 4;
  q.px = q.blk.x0 + 4 * (q.quad & 1) + (l & 3);
  q.py = q.blk.y0 + 4 * (q.quad >> 1) + ((l >> 2) & 3);
  q.inside = q.px < Rr.W && q.py < Rr.H;
  q.fpx = (float)q.px;
  q.fpy = (float)q.py;
  q.p = (int64_t)q.py * Rr.W + q.px;
  q.off = (int64_t)q.view * Rr.W * Rr.H;
  return q;
}

// Can the record reach alpha >= alpha_min anywhere in the block? alpha = o 2^p
// with p = pa dx^2 + pb dx dy + pc dy^2 <= 0 (pa, pc < 0), so it needs
// max over the block of p >= log2(alpha_min / o). If the centre lies in the
// block the maximum is 0; otherwise it lies on the block edge(s) facing the
// centre, where p restricted to the edge is a 1D concave quadratic whose
// maximiser is clamped to the edge. The continuous block contains every pixel
// centre, and the threshold carries a margin of 1e-3 (FP32 rounding of p is
// ~1e-6), so a skipped record has alpha < alpha_min at every pixel: the
// result cannot change, only the work.
__device__ __forceinline__ bool ellipse_meets(const float4& g, const float4& cb, const Block& s, float log2_amin) {
  const float u = g.x, v = g.y, pa = g.z, pb = g.w, pc = cb.x;
  const float thr = log2_amin - __builtin_amdgcn_logf(cb.y) - 1e-3f;  // log2(alpha_min / o)
  const float X0 = (float)s.x0, X1 = (float)s.x1, Y0 = (float)s.y0, Y1 = (float)s.y1;
  const float cx = fminf(fmaxf(u, X0), X1), cy = fminf(fmaxf(v, Y0), Y1);
  float best = (cx == u && cy == v) ? 0.f : -INFINITY;
  if (cx != u) {  // edge x = cx: maximise over y
    const float dX = cx - u;
    const float y = fminf(fmaxf(v - pb * dX * __builtin_amdgcn_rcpf(2.f * pc), Y0), Y1);
    const float dy = y - v;
    best = fmaxf(best, fmaf(pa * dX, dX, fmaf(pb * dX, dy, pc * dy * dy)));
  }
  if (cy != v) {  // edge y = cy: maximise over x
    const float dY = cy - v;
    const float x = fminf(fmaxf(u - pb * dY * __builtin_amdgcn_rcpf(2.f * pa), X0), X1);
    const float dx = x - u;
    best = fmaxf(best, fmaf(pa * dx, dx, fmaf(pb * dx, dY, pc * dY * dY)));
  }
  return best >= thr;
}

// Quadrants of the block (bit k = quadrant k, row-major) the record may reach:
// the packed support box (x0 | x1 << 16, y0 | y1 << 16) must meet the block
// and, if EXACT, the record must pass the ellipse test on the block; a
// quadrant must also meet the support box.
template <bool EXACT>
__device__ __forceinline__ uint32_t quad_mask(const float4& g, const float4& cb, const Block& s, float log2_amin) {
  const uint32_t bx = __float_as_uint(cb.z), by = __float_as_uint(cb.w);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16), y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  bool meets = (x0 <= s.x1) & (x1 >= s.x0) & (y0 <= s.y1) & (y1 >= s.y0);  // no short-circuit branches
  if (EXACT) meets = meets && ellipse_meets(g, cb, s, log2_amin);
  const uint32_t L = x0 <= s.x0 + 3, R = x1 >= s.x0 + 4, T = y0 <= s.y0 + 3, B = y1 >= s.y0 + 4;
  const uint32_t m = (L & T) | ((R & T) << 1) | ((L & B) << 2) | ((R & B) << 3);
  return meets ? m : 0u;
}

// Can the record reach alpha >= alpha_min anywhere in the block (support box,
// then the ellipse test)?
__device__ __forceinline__ bool block_meets(const float4& g, const float4& cb, const Block& s, float log2_amin) {
  const uint32_t bx = __float_as_uint(cb.z), by = __float_as_uint(cb.w);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16), y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  return ((x0 <= s.x1) & (x1 >= s.x0) & (y0 <= s.y1) & (y1 >= s.y0)) && ellipse_meets(g, cb, s, log2_amin);
}

__device__ __forceinline__ bool box_holds(float fbx, float fby, int px, int py) {
  const uint32_t bx = __float_as_uint(fbx), by = __float_as_uint(fby);
  return (px >= (int)(bx & 0xffffu)) & (px <= (int)(bx >> 16)) & (py >= (int)(by & 0xffffu)) & (py <= (int)(by >> 16));
}

// Lanes whose bit is set in the wave-uniform mask m append `val` to `list`
// after its first `len` entries, in lane order.
__device__ __forceinline__ void list_append(uint16_t* list, int len, uint64_t m, int lane, int val) {
  if ((m >> lane) & 1ull) {
    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    list[len + below] = (uint16_t)val;
  }
}

// The float4 at byte offset `boff` of an LDS array.
__device__ __forceinline__ float4 lds_at(const float4* arr, int boff) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(arr) + boff);
}

struct FwdSmem {
  static constexpr int kBatch = kFwdBatch, kDummy = kFwdBatch;
  float4 uvab[kBatch + 1];
  float4 cob[kBatch + 1];
  float4 rgbz[kBatch + 1];
  uint16_t list[kWavesPerTile][4][kListCap + 4];
};

// Backward, block walk: the batch's records and their Gaussian ids.
struct BwdSmem {
  static constexpr int kBatch = kBwdBatch;
  float4 uvab[kBatch];
  float4 cob[kBatch];
  float4 rgbz[kBatch];
  uint32_t gid[kBatch];
  int max_last;
};

// Backward, quadrant walk (six fields): the batch's records (and the all-zero
// record), their Gaussian ids, six per-Gaussian partial sums per record (zero
// between batches) and one visit list per (wave, quadrant).
struct QuadSmem {
  static constexpr int kBatch = kQuadBatch, kDummy = kQuadBatch, kNF = 6;
  float4 uvab[kBatch + 1];
  float4 cob[kBatch + 1];
  float4 rgbz[kBatch + 1];
  float acc[kBatch * kNF];
  uint32_t gid[kBatch];
  uint16_t list[kWavesPerTile][4][kListCap + 4];
  int max_last;
};

// The all-zero record; written once per workgroup before its first barrier.
__device__ __forceinline__ void init_smem(FwdSmem& sm) {
  if (threadIdx.x == 0) {
    sm.uvab[FwdSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
    sm.cob[FwdSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
    sm.rgbz[FwdSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// STATS = true: instead of writing outputs, count the algorithmic work (for the
// benchmark's roofline): pairs whose pixel lies in the Gaussian's support box
// before the pixel stops, and pairs composited. The lists then come from the
// support boxes alone, so every such pair is visited.
template <bool STATS>
__device__ __forceinline__ void fwd_item(const Raster& Rr, const FwdArgs& a, int item, FwdSmem& sm) {
  constexpr int kBatch = FwdSmem::kBatch, kDummy = FwdSmem::kDummy;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Pixel q = item_pixel(Rr, item);
  const int2 rg = a.ranges[item];
  const int start = rg.x, end = rg.y;
  // T > 0: the lane is compositing; T < 0: it has stopped and -T is its final
  // transmittance (T >= T_min > 0 while compositing, so the sign is free).
  float T = q.inside ? 1.f : -1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  int last16 = 0;  // 16 x (list position of the last composited Gaussian + 1)
  uint32_t n_eval = 0, n_comp = 0;
  const uint16_t* mylist = sm.list[w][q.quad];

  for (int base = start; base < end; base += kBatch) {
    if (__syncthreads_count(T > 0.f) == 0) break;
#pragma unroll
    for (int h = 0; h < (kBatch + kTileThreads - 1) / kTileThreads; ++h) {
      const int sl = h * kTileThreads + tid, i = base + sl;
      if (sl < kBatch && i < end) {
        const uint32_t gid = a.ids[i];
        sm.uvab[sl] = a.rec_uvab[kRec * gid];
        sm.cob[sl] = a.rec_cob[kRec * gid];
        sm.rgbz[sl] = a.rec_rgbz[kRec * gid];
      }
    }
    __syncthreads();
    const int cnt = min(kBatch, end - base);
    const int nch = (cnt + kWave - 1) / kWave;
    int k = 0;
    while (k < nch) {
      // one segment: append chunks to the quadrant lists until one would overflow
      const uint64_t alive = __ballot(T > 0.f);
      if (alive == 0) break;
      int len0 = 0, len1 = 0, len2 = 0, len3 = 0;
      for (; k < nch; ++k) {
        const int r = k * kWave + lane;
        const uint32_t qm = r < cnt ? quad_mask<!STATS>(sm.uvab[r], sm.cob[r], q.blk, Rr.log2_amin) : 0u;
        // a quadrant whose lanes have all stopped takes no entries
        const uint64_t m0 = (alive & 0xffffull) ? __ballot(qm & 1u) : 0ull;
        const uint64_t m1 = (alive & 0xffff0000ull) ? __ballot(qm & 2u) : 0ull;
        const uint64_t m2 = (alive & 0xffff00000000ull) ? __ballot(qm & 4u) : 0ull;
        const uint64_t m3 = (alive & 0xffff000000000000ull) ? __ballot(qm & 8u) : 0ull;
        const int c0 = __popcll(m0), c1 = __popcll(m1), c2 = __popcll(m2), c3 = __popcll(m3);
        if (len0 + c0 > kListCap || len1 + c1 > kListCap || len2 + c2 > kListCap || len3 + c3 > kListCap) break;
        // entries are LDS byte offsets of the slot inside each record array
        list_append(sm.list[w][0], len0, m0, lane, 16 * r);
        list_append(sm.list[w][1], len1, m1, lane, 16 * r);
        list_append(sm.list[w][2], len2, m2, lane, 16 * r);
        list_append(sm.list[w][3], len3, m3, lane, 16 * r);
        len0 += c0;
        len1 += c1;
        len2 += c2;
        len3 += c3;
      }
      const int myl = q.quad == 0 ? len0 : (q.quad == 1 ? len1 : (q.quad == 2 ? len2 : len3));
      const int maxl = __builtin_amdgcn_readfirstlane(max(max(len0, len1), max(len2, len3)));
      // (list position + 1) * 16 of slot 0: last16 = code + byte offset
      const int code = 16 * (base - start + 1);
      __builtin_amdgcn_wave_barrier();
      // One step per record of the row's list. Every lane runs the same
      // instructions: a skipped pair (alpha < alpha_min, or the all-zero
      // record) acts as alpha = 0; a stopped lane has T < 0, so its Tn <
      // T_min and it adds w = 0 and keeps T.
      auto step = [&](const float4& g, const float4& cb, const float4& cz, int jb) {
        const PairEval pe = eval_pair(q.fpx - g.x, q.fpy - g.y, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
        if (STATS && T > 0.f && jb != 16 * kDummy && box_holds(cb.z, cb.w, q.px, q.py)) ++n_eval;
        const float al = pe.use ? pe.alpha : 0.f;
        const float Tn = T * (1.f - al);
        const bool comp = Tn >= Rr.tmin;  // false for a stopped lane and at the stop
        const float wt = comp ? al * T : 0.f;
        C0 = fmaf(cz.x, wt, C0);
        C1 = fmaf(cz.y, wt, C1);
        C2 = fmaf(cz.z, wt, C2);
        D = fmaf(cz.w, wt, D);
        last16 = (comp && pe.use) ? code + jb : last16;
        if (STATS && comp && pe.use) ++n_comp;
        T = comp ? Tn : -fabsf(T);
      };
      // walk while some lane is compositing and its row's list has not ended
      auto going = [&](int t) { return (t < maxl) & ((__ballot(T > 0.f) & __ballot(t < myl)) != 0); };
      // Software pipeline, unrolled by two so that no record is copied
      // between registers: while step t runs on one record set, the other
      // set receives the record of step t + 1 from LDS, and the list entry of
      // step t + 2 is read (entries past the row's list end are not used).
      // The walk condition is checked before every second step only: a step
      // after it turned false is a no-op (every lane has stopped, or every
      // row reads the all-zero record), and entries up to kListCap + 2 exist
      // for its reads. The loop is tested at its end (one exit) and the test
      // itself has no branch, so the body is one basic block and the carried
      // sums stay in the same registers around it.
      int jA = 0 < myl ? mylist[0] : 16 * kDummy;
      int jn = mylist[1];
      float4 gA = lds_at(sm.uvab, jA), cbA = lds_at(sm.cob, jA), czA = lds_at(sm.rgbz, jA);
      if (going(0)) {
        int t = 0;
        do {
          const int jB = t + 1 < myl ? jn : 16 * kDummy;
          jn = mylist[t + 2];
          const float4 gB = lds_at(sm.uvab, jB), cbB = lds_at(sm.cob, jB), czB = lds_at(sm.rgbz, jB);
          step(gA, cbA, czA, jA);
          ++t;
          jA = t + 1 < myl ? jn : 16 * kDummy;
          jn = mylist[t + 2];
          gA = lds_at(sm.uvab, jA);
          cbA = lds_at(sm.cob, jA);
          czA = lds_at(sm.rgbz, jA);
          step(gB, cbB, czB, jB);
          ++t;
        } while (going(t));
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (STATS) {
    unsigned long long e = n_eval, cm = n_comp;
    for (int o = 32; o > 0; o >>= 1) {
      e += __shfl_xor(e, o, 64);
      cm += __shfl_xor(cm, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&a.stats[0], e);
      atomicAdd(&a.stats[1], cm);
    }
    return;
  }
  if (q.inside) {
    T = fabsf(T);
    const int64_t P = (int64_t)Rr.W * Rr.H;
    const int64_t p = q.off + q.p;
    float* col = a.color + 3 * q.off;
    col[q.p] = fmaf(T, Rr.bg0, C0);
    col[P + q.p] = fmaf(T, Rr.bg1, C1);
    col[2 * P + q.p] = fmaf(T, Rr.bg2, C2);
    a.depth[p] = D;
    a.alpha[p] = 1.f - T;
    a.Tfin[p] = T;
    a.last[p] = last16 >> 4;
  }
}

// Quadrants of the block (bit k = quadrant k, row-major) where the record can
// reach alpha >= alpha_min: its support box meets the quadrant and the
// ellipse test passes on the quadrant itself.
__device__ __forceinline__ uint32_t quad_mask_exact(const float4& g, const float4& cb, const Block& s,
                                                    float log2_amin) {
  const uint32_t bx = __float_as_uint(cb.z), by = __float_as_uint(cb.w);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16), y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Block qb;
    qb.x0 = s.x0 + 4 * (k & 1);
    qb.x1 = qb.x0 + 3;
    qb.y0 = s.y0 + 4 * (k >> 1);
    qb.y1 = qb.y0 + 3;
    if ((x0 <= qb.x1) & (x1 >= qb.x0) & (y0 <= qb.y1) & (y1 >= qb.y0))
      m |= ellipse_meets(g, cb, qb, log2_amin) ? (1u << k) : 0u;
  }
  return m;
}

// Lanes whose bit is set in the wave-uniform mask m (c bits) append `val` to
// `list` after its first `len` entries, highest lane first.
__device__ __forceinline__ void list_append_desc(uint16_t* list, int len, uint64_t m, int c, int lane, int val) {
  if ((m >> lane) & 1ull) {
    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    list[len + c - 1 - below] = (uint16_t)val;
  }
}

// Maximum over the lane's 16-lane row.
__device__ __forceinline__ int row_max_int(int v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Sums of six per-lane partials (fields 0-4 and 9, numbered 0-5) over each
// 16-lane row. Field-splitting: at each exchange a lane keeps half of its
// fields and hands the other half to its partner (row_mirror pairs lane bit
// 3, row_half_mirror bit 2, quad_perm [2,3,0,1] bit 1), then the pair across
// bit 0 is summed: lanes (b3 b2 b1 b0) with b0 = 0 and 2 b2 + b1 <= 2 end
// with field 3 b3 + 2 b2 + b1. Returns the lane's sum and sets *f to its
// field, or -1.
__device__ __forceinline__ float row_reduce6(const float v[10], int lane, int* f) {
  const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
  const float w6[6] = {v[0], v[1], v[2], v[3], v[4], v[9]};
  float r[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = (b3 ? w6[3 + k] : w6[k]) + dpp_f<0x140>(b3 ? w6[k] : w6[3 + k]);  // row_mirror
  r[3] = 0.f;
  float s[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) s[k] = (b2 ? r[2 + k] : r[k]) + dpp_f<0x141>(b2 ? r[k] : r[2 + k]);  // row_half_mirror
  float t = (b1 ? s[1] : s[0]) + dpp_f<0x4e>(b1 ? s[0] : s[1]);  // quad_perm [2,3,0,1]
  t += dpp_f<0xb1>(t);                                          // quad_perm [1,0,3,2]
  const int loc = 2 * (int)b2 + (int)b1;
  *f = (!b0 && loc <= 2) ? 3 * (int)b3 + loc : -1;
  return t;
}

// Column of the [n, 10] gradient sums that field f of the six-field
// reduction adds to.
__device__ __forceinline__ int g2d_field6(int f) { return f < 5 ? f : 9; }

// Per-pixel state of the backward: the forward's final transmittance and last
// composited position, the upstream gradients, and the running suffix term.
struct BwdPix {
  float T, g0, g1, g2, gd, gS, gA;
  int last;
};

// dL/dalpha_j = T_j (g . c_j) - (g . S_j + ga T_fin) / (1 - alpha_j) with the
// suffix sums S_j = sum_{u > j} c_u alpha_u T_u + T_fin bg (colour) and
// sum_{u > j} z_u alpha_u T_u (depth), g = (gC, gD). Only the dot product
// gS = g . S_j is needed; the background enters it through T_fin bg.
__device__ __forceinline__ BwdPix bwd_pixel(const Raster& Rr, const BwdArgs& a, const Pixel& q) {
  BwdPix b{1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0};
  float ga = 0.f;
  if (q.inside) {
    const int64_t P = (int64_t)Rr.W * Rr.H;
    const int64_t p = q.off + q.p;
    const float* gC = a.gC + 3 * q.off;
    b.T = a.Tfin[p];
    b.last = a.last[p];
    b.g0 = gC[q.p];
    b.g1 = gC[P + q.p];
    b.g2 = gC[2 * P + q.p];
    b.gd = a.gD[p];
    ga = a.gA ? a.gA[p] : 0.f;
  }
  b.gS = b.T * (b.g0 * Rr.bg0 + b.g1 * Rr.bg1 + b.g2 * Rr.bg2);
  b.gA = ga * b.T;
  return b;
}

// One pair of the back-to-front walk: recomputes T_j, advances the suffix
// term and writes the ten per-pair partials (sums of q (dx, dy, dx^2, dx dy,
// dy^2) with q = dL/dp / ln 2 for alpha = o 2^p, then d alpha / d o times
// dL/dalpha, colour, direct depth). A lane without a hit runs the same
// instructions with alpha = 0: its transmittance and suffix term are
// unchanged and its partials are 0.
__device__ __forceinline__ void bwd_pair(BwdPix& b, const PairEval& pe, bool hit, float dx, float dy,
                                         const float4& cz, float v[10]) {
  const float al = hit ? pe.alpha : 0.f;
  const float inv = __builtin_amdgcn_rcpf(1.f - al);  // 1 ulp; alpha <= alpha_max < 1
  const float Tj = b.T * inv;
  const float wt = al * Tj;
  v[6] = wt * b.g0;
  v[7] = wt * b.g1;
  v[8] = wt * b.g2;
  v[9] = wt * b.gd;
  const float gc = fmaf(b.g0, cz.x, fmaf(b.g1, cz.y, fmaf(b.g2, cz.z, b.gd * cz.w)));
  const float dA = fmaf(Tj, gc, -inv * (b.gS - b.gA));
  b.gS = fmaf(gc, wt, b.gS);
  b.T = Tj;
  // a clamped alpha does not depend on o or sigma
  const float dAs = (hit && !pe.clamped) ? dA : 0.f;
  v[5] = dAs * pe.e;  // d alpha / d o = exp(-sigma)
  // the projection backward turns the sums of q (dx, dy, dx^2, dx dy, dy^2)
  // into dL/d(u, v) and the conic terms
  const float gp = dAs * pe.alpha;
  const float gpx = gp * dx, gpy = gp * dy;
  v[0] = gpx;
  v[1] = gpy;
  v[2] = gpx * dx;
  v[3] = gpx * dy;
  v[4] = gpy * dy;
}

// Backward of one item, block walk (all ten fields: mapping). Each wave walks
// the records that can reach its 8x8 block (support box, then the ellipse
// test) back to front from the largest `last` of its pixels, one record per
// step with the record broadcast from LDS; a wave's sums of a record's ten
// partials come from a field-splitting butterfly and go to the [n, 10]
// gradient sums with one 10-lane atomic (DET: they are stored at (list
// position, wave) of a.part, and the wave's bit set in a.mask).
template <bool DET>
__device__ __forceinline__ void bwd_item_block(const Raster& Rr, const BwdArgs& a, int item, BwdSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Pixel q = item_pixel(Rr, item);
  BwdPix b = bwd_pixel(Rr, a, q);
  __syncthreads();  // the previous item (persistent launch) is done with max_last
  if (tid == 0) sm.max_last = 0;
  __syncthreads();
  if (b.last > 0) atomicMax(&sm.max_last, b.last);
  const int wmax = wave_max_int(b.last);
  __syncthreads();
  const int bmax = sm.max_last;
  const int start = a.ranges[item].x;

  constexpr int kBatch = BwdSmem::kBatch;
  for (int bend = start + bmax; bend > start; bend -= kBatch) {
    const int bstart = max(start, bend - kBatch);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < (kBatch + kTileThreads - 1) / kTileThreads; ++h) {
      const int sl = h * kTileThreads + tid, i = bstart + sl;
      if (sl < kBatch && i < bend) {
        const uint32_t gid = a.ids[i];
        sm.gid[sl] = gid;
        sm.uvab[sl] = a.rec_uvab[kRec * gid];
        sm.cob[sl] = a.rec_cob[kRec * gid];
        sm.rgbz[sl] = a.rec_rgbz[kRec * gid];
      }
    }
    __syncthreads();
    const int cnt = min(bend, start + wmax) - bstart;  // records this wave may need
    for (int c = (cnt - 1) >> 6; c >= 0; --c) {
      const int r = c * kWave + lane;
      bool meets = false;
      if (r < cnt) {
        const float4 cb = sm.cob[r];
        meets = block_meets(sm.uvab[r], cb, q.blk, Rr.log2_amin);
      }
      uint64_t m = __ballot(meets);
      const int cbase = __builtin_amdgcn_readfirstlane(c * kWave);  // keep the index arithmetic scalar
      // one visit: the record at slot li (its three float4s already in registers)
      auto visit = [&](const float4& g, const float4& cb, const float4& cz, int li) {
        const int pos = bstart + li - start;
        const float dx = q.fpx - g.x, dy = q.fpy - g.y;
        const PairEval pe = eval_pair(dx, dy, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
        const bool hit = pos < b.last && pe.use;
        if (!__any(hit)) return;
        float v[10];
        bwd_pair(b, pe, hit, dx, dy, cz, v);
        int f;
        const float u = wave_reduce10(v, lane, &f);
        if (DET) {
          const int64_t slot = bstart + li;  // position in the ids array
          if (f >= 0) a.part[(slot * 16 + w) * 10 + f] = u;
          if (lane == 0) atomicOr(a.mask + slot, 1u << w);
        } else if (f >= 0) {
          atomicAdd(a.g2d + 10 * (int64_t)sm.gid[li] + f, u);
        }
      };
      // the highest remaining record of the mask (removed from it)
      auto take = [&]() {
        const int bit = 63 - __builtin_clzll(m);
        m &= ~(1ull << bit);
        return cbase + bit;
      };
      // Software pipeline, unrolled by two: the next visit's record is read
      // from LDS while the current one is evaluated, into the other register
      // set, so no record is copied between registers.
      if (m == 0) continue;
      int lA = take();
      float4 gA = sm.uvab[lA], cbA = sm.cob[lA], czA = sm.rgbz[lA];
      for (;;) {
        const bool moreB = m != 0;
        int lB = 0;
        float4 gB, cbB, czB;
        if (moreB) {
          lB = take();
          gB = sm.uvab[lB];
          cbB = sm.cob[lB];
          czB = sm.rgbz[lB];
        }
        visit(gA, cbA, czA, lA);
        if (!moreB) break;
        const bool moreA = m != 0;
        if (moreA) {
          lA = take();
          gA = sm.uvab[lA];
          cbA = sm.cob[lA];
          czA = sm.rgbz[lA];
        }
        visit(gB, cbB, czB, lB);
        if (!moreA) break;
      }
    }
  }
}

// Backward of one item, quadrant walk (the six fields of a pose-only
// backward: tracking). Each wave walks its 8x8 block back to front from the
// largest `last` of its pixels; per batch of records staged in LDS, each of
// its four rows (4x4 quadrants) gets a visit list of the records that can
// reach alpha >= alpha_min in the quadrant (support box and ellipse test on
// the quadrant) at a position before the quadrant's largest `last`, in
// descending position; the rows walk their lists side by side, a row whose
// list has ended reading the all-zero record. A row's sums of a record's six
// partials are added to the record's accumulator in LDS; after the batch the
// workgroup adds every non-zero accumulator to the [n, 10] gradient sums (one
// global atomic per (Gaussian, tile, field)). On the 640 x 480 tracking frame
// this beats the block walk (smaller Gaussians on screen leave more of a
// block's quadrants untouched); with ten fields on the 1200 x 680 mapping
// frame the block walk is faster (its lists are hardly longer than the
// quadrants', and its butterfly serves 64 lanes per record).
//
// DET: instead of the LDS accumulators, each row stores its sums of a record
// to a.part at (list position of the record, quadrant of the tile) and sets
// that quadrant's bit in a.mask; a later pass adds them per Gaussian in a
// fixed order, so the result does not depend on the order rows and
// workgroups run in.
template <bool DET>
__device__ __forceinline__ void bwd_item_quad(const Raster& Rr, const BwdArgs& a, int item, QuadSmem& sm) {
  constexpr int kBatch = QuadSmem::kBatch, kDummy = QuadSmem::kDummy, NF = QuadSmem::kNF;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Pixel q = item_pixel(Rr, item);
  BwdPix b = bwd_pixel(Rr, a, q);
  __syncthreads();  // the previous item (persistent launch) is done with max_last
  if (tid == 0) sm.max_last = 0;
  __syncthreads();
  if (b.last > 0) atomicMax(&sm.max_last, b.last);
  // the largest `last` of each quadrant (row), wave-uniform
  const int rl = row_max_int(b.last);
  const int ql0 = __builtin_amdgcn_readlane(rl, 0), ql1 = __builtin_amdgcn_readlane(rl, 16);
  const int ql2 = __builtin_amdgcn_readlane(rl, 32), ql3 = __builtin_amdgcn_readlane(rl, 48);
  const int wmax = max(max(ql0, ql1), max(ql2, ql3));
  __syncthreads();
  const int bmax = sm.max_last;
  const int start = a.ranges[item].x;
  const uint16_t* mylist = sm.list[w][q.quad];

  for (int bend = start + bmax; bend > start; bend -= kBatch) {
    const int bstart = max(start, bend - kBatch);
    const int boff = bstart - start;  // list position of slot 0
    __syncthreads();  // the previous batch's flush is done with gid and acc
#pragma unroll
    for (int h = 0; h < (kBatch + kTileThreads - 1) / kTileThreads; ++h) {
      const int sl = h * kTileThreads + tid, i = bstart + sl;
      if (sl < kBatch && i < bend) {
        const uint32_t gid = a.ids[i];
        sm.gid[sl] = gid;
        sm.uvab[sl] = a.rec_uvab[kRec * gid];
        sm.cob[sl] = a.rec_cob[kRec * gid];
        sm.rgbz[sl] = a.rec_rgbz[kRec * gid];
      }
    }
    __syncthreads();
    const int cnt = min(bend, start + wmax) - bstart;  // records this wave may need
    int k = cnt > 0 ? (cnt - 1) >> 6 : -1;
    while (k >= 0) {
      // one segment: append chunks (back to front) to the quadrant lists until one would overflow
      int len0 = 0, len1 = 0, len2 = 0, len3 = 0;
      for (; k >= 0; --k) {
        const int r = k * kWave + lane;
        const int pos = boff + r;
        const uint32_t qm = r < cnt ? quad_mask_exact(sm.uvab[r], sm.cob[r], q.blk, Rr.log2_amin) : 0u;
        const uint64_t m0 = __ballot((qm & 1u) && pos < ql0);
        const uint64_t m1 = __ballot((qm & 2u) && pos < ql1);
        const uint64_t m2 = __ballot((qm & 4u) && pos < ql2);
        const uint64_t m3 = __ballot((qm & 8u) && pos < ql3);
        const int c0 = __popcll(m0), c1 = __popcll(m1), c2 = __popcll(m2), c3 = __popcll(m3);
        if (len0 + c0 > kListCap || len1 + c1 > kListCap || len2 + c2 > kListCap || len3 + c3 > kListCap) break;
        // entries are LDS byte offsets of the slot inside each record array
        list_append_desc(sm.list[w][0], len0, m0, c0, lane, 16 * r);
        list_append_desc(sm.list[w][1], len1, m1, c1, lane, 16 * r);
        list_append_desc(sm.list[w][2], len2, m2, c2, lane, 16 * r);
        list_append_desc(sm.list[w][3], len3, m3, c3, lane, 16 * r);
        len0 += c0;
        len1 += c1;
        len2 += c2;
        len3 += c3;
      }
      const int myl = q.quad == 0 ? len0 : (q.quad == 1 ? len1 : (q.quad == 2 ? len2 : len3));
      const int maxl = __builtin_amdgcn_readfirstlane(max(max(len0, len1), max(len2, len3)));
      __builtin_amdgcn_wave_barrier();
      // one step per record of the row's list (pend: the row's list has not ended)
      auto step = [&](const float4& g, const float4& cb, const float4& cz, int jb, bool pend) {
        const float dx = q.fpx - g.x, dy = q.fpy - g.y;
        const PairEval pe = eval_pair(dx, dy, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
        const bool hit = boff + (jb >> 4) < b.last && pe.use;  // the all-zero record never passes `use`
        float v[10];
        bwd_pair(b, pe, hit, dx, dy, cz, v);
        int f;
        const float u = row_reduce6(v, lane, &f);
        if (DET) {
          if (__ballot(hit) != 0) {
            const int64_t slot = bstart + (jb >> 4);  // position in the ids array
            const int quad = 4 * w + q.quad;          // quadrant of the tile
            if (pend && f >= 0) a.part[(slot * 16 + quad) * NF + f] = u;
            if (pend && (lane & 15) == 0) atomicOr(a.mask + slot, 1u << quad);
          }
        } else if (pend && f >= 0) {
          atomicAdd(sm.acc + NF * (jb >> 4) + f, u);
        }
      };
      // Software pipeline, unrolled by two so that no record is copied
      // between registers: while step t runs on one record set, the other
      // set receives the record of step t + 1 from LDS, and the list entry of
      // step t + 2 is read (entries past the row's list end are not used).
      // The loop is tested at its end only, so with an odd maxl its last
      // step runs past every row's list: a no-op (the all-zero record, no
      // accumulation), and entries up to kListCap + 2 exist for its reads.
      int jA = 0 < myl ? mylist[0] : 16 * kDummy;
      int jn = mylist[1];
      float4 gA = lds_at(sm.uvab, jA), cbA = lds_at(sm.cob, jA), czA = lds_at(sm.rgbz, jA);
      if (0 < maxl) {
        int t = 0;
        do {
          const int jB = t + 1 < myl ? jn : 16 * kDummy;
          jn = mylist[t + 2];
          const float4 gB = lds_at(sm.uvab, jB), cbB = lds_at(sm.cob, jB), czB = lds_at(sm.rgbz, jB);
          step(gA, cbA, czA, jA, t < myl);
          ++t;
          jA = t + 1 < myl ? jn : 16 * kDummy;
          jn = mylist[t + 2];
          gA = lds_at(sm.uvab, jA);
          cbA = lds_at(sm.cob, jA);
          czA = lds_at(sm.rgbz, jA);
          step(gB, cbB, czB, jB, t < myl);
          ++t;
        } while (t < maxl);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (DET) continue;
    __syncthreads();  // every row's sums of this batch are in acc
    for (int i = tid; i < (bend - bstart) * NF; i += kTileThreads) {
      const float val = sm.acc[i];
      if (val != 0.f) {
        const int slot = i / NF, f = i - slot * NF;
        atomicAdd(a.g2d + 10 * (int64_t)sm.gid[slot] + g2d_field6(f), val);
        sm.acc[i] = 0.f;
      }
    }
  }
}

// The all-zero record and zero accumulators; written before the first barrier.
__device__ __forceinline__ void init_smem(QuadSmem& sm) {
  if (threadIdx.x == 0) {
    sm.uvab[QuadSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
    sm.cob[QuadSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
    sm.rgbz[QuadSmem::kDummy] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int i = threadIdx.x; i < QuadSmem::kBatch * QuadSmem::kNF; i += kTileThreads) sm.acc[i] = 0.f;
}

template <bool STATS>
__global__ __launch_bounds__(kTileThreads) void k_render_fwd(Raster Rr, FwdArgs a) {
  __shared__ FwdSmem sm;
  init_smem(sm);
  fwd_item<STATS>(Rr, a, xcd_tile(blockIdx.x, gridDim.x), sm);
}

template <bool DET>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd_block(Raster Rr, BwdArgs a) {
  __shared__ BwdSmem sm;
  bwd_item_block<DET>(Rr, a, xcd_tile(blockIdx.x, gridDim.x), sm);
}

template <bool DET>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd_quad(Raster Rr, BwdArgs a) {
  __shared__ QuadSmem sm;
  init_smem(sm);
  bwd_item_quad<DET>(Rr, a, xcd_tile(blockIdx.x, gridDim.x), sm);
}

// Persistent workgroups: take the next item from the queue until it is empty.
// Every workgroup reaches the exit once the counter passes n_items.
__device__ __forceinline__ int next_item(int* queue, const int* order, int n_items, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
  __syncthreads();
  const int qi = *s_item;
  if (qi >= n_items) return -1;
  return order ? order[qi] : qi;
}

__global__ __launch_bounds__(kTileThreads) void k_render_fwd_persistent(Raster Rr, FwdArgs a) {
  __shared__ FwdSmem sm;
  __shared__ int s_item;
  init_smem(sm);
  for (;;) {
    const int item = next_item(a.queue, a.order, a.n_items, &s_item);
    if (item < 0) break;
    fwd_item<false>(Rr, a, item, sm);
  }
}

template <bool DET>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd_block_persistent(Raster Rr, BwdArgs a) {
  __shared__ BwdSmem sm;
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(a.queue, a.order, a.n_items, &s_item);
    if (item < 0) break;
    bwd_item_block<DET>(Rr, a, item, sm);
  }
}

template <bool DET>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd_quad_persistent(Raster Rr, BwdArgs a) {
  __shared__ QuadSmem sm;
  __shared__ int s_item;
  init_smem(sm);
  for (;;) {
    const int item = next_item(a.queue, a.order, a.n_items, &s_item);
    if (item < 0) break;
    bwd_item_quad<DET>(Rr, a, item, sm);
  }
}

// Deterministic backward, before the compositing pass: rev[goff[o] + j] =
// list position of record o in the j-th tile of its tile rectangle (row-major),
// where goff is the exclusive scan of the records' tile counts.
__global__ __launch_bounds__(256) void k_det_rev(Raster Rr, const int2* __restrict__ ranges,
                                               const uint32_t* __restrict__ ids, const int4* __restrict__ rect,
                                               const uint32_t* __restrict__ goff, uint32_t* __restrict__ rev) {
  const int item = blockIdx.x;
  const int tile = item % Rr.n_tiles;
  const int ty = tile / Rr.ntx, tx = tile - ty * Rr.ntx;
  const int2 rg = ranges[item];
  for (int i = rg.x + (int)threadIdx.x; i < rg.y; i += blockDim.x) {
    const uint32_t o = ids[i];
    const int4 r = rect[o];
    const int tx0 = r.x & 0xffff, tx1 = (int)((uint32_t)r.x >> 16), ty0 = r.y & 0xffff;
    rev[goff[o] + (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0))] = (uint32_t)i;
  }
}

// Deterministic backward, after the compositing pass: one thread per (record,
// field) adds the stored quadrant sums of its tiles (tiles in row-major order
// of the record's rectangle, quadrants in order) and stores the total into
// the [n, 10] gradient sums.
template <int NF>
__global__ __launch_bounds__(256) void k_det_reduce(const int4* __restrict__ rect, const uint32_t* __restrict__ goff,
                                                  const uint32_t* __restrict__ rev, const uint32_t* __restrict__ mask,
                                                  const float* __restrict__ part, int64_t n_rec,
                                                  float* __restrict__ g2d) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_rec * NF) return;
  const int64_t o = idx / NF;
  const int f = (int)(idx - o * NF);
  const int cnt = rect[o].w;
  if (cnt == 0) return;
  const uint32_t b = goff[o];
  float sum = 0.f;
  for (int j = 0; j < cnt; ++j) {
    const int64_t slot = rev[b + j];
    uint32_t m = mask[slot];
    while (m) {
      const int quad = __builtin_ctz(m);
      m &= m - 1u;
      sum += part[(slot * 16 + quad) * NF + f];
    }
  }
  g2d[10 * o + (NF == 10 ? f : g2d_field6(f))] = sum;
}

// Support-box pairs before each pixel's last composited Gaussian: the pairs
// the backward must evaluate (work counter; reads the forward's `last`).
__global__ __launch_bounds__(kTileThreads) void k_count_bwd_pairs(Raster Rr, FwdArgs a) {
  __shared__ float4 s_cob[kTileThreads];
  const int item = blockIdx.x;
  const Pixel q = item_pixel(Rr, item);
  const int last = q.inside ? a.last[q.off + q.p] : 0;
  const int2 rg = a.ranges[item];
  unsigned long long n = 0;
  for (int base = rg.x; base < rg.y; base += kTileThreads) {
    __syncthreads();
    if (base + (int)threadIdx.x < rg.y) s_cob[threadIdx.x] = a.rec_cob[kRec * a.ids[base + threadIdx.x]];
    __syncthreads();
    const int cnt = min(kTileThreads, rg.y - base);
    for (int j = 0; j < cnt; ++j)
      if (base - rg.x + j < last && box_holds(s_cob[j].z, s_cob[j].w, q.px, q.py)) ++n;
  }
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(&a.stats[2], n);
}

// Longest-list-first item order: bucket items by floor(log2(len + 1)) and
// emit the buckets from the longest down (order inside a bucket is arbitrary).
// Each wave aggregates its items per bucket (one leader lane per distinct
// bucket), so the 32 global counters see one atomic per (wave, bucket)
// instead of one per item.
__device__ __forceinline__ int order_bucket(const int2* __restrict__ ranges, int i) {
  const int2 r = ranges[i];
  return 31 - __clz(r.y - r.x + 1);
}

__global__ void k_order_hist(const int2* __restrict__ ranges, int n_items, int* __restrict__ temp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n_items;
  const int b = valid ? order_bucket(ranges, i) : -1;
  uint64_t remaining = __ballot(valid);
  while (remaining) {
    const int leader = __builtin_ctzll(remaining);
    const int lb = __shfl(b, leader, 64);
    const uint64_t same = __ballot(valid && b == lb);
    if (lane == leader) atomicAdd(&temp[lb], __popcll(same));
    remaining &= ~same;
  }
}

__global__ void k_order_scan(int* temp) {
  if (threadIdx.x != 0) return;
  int s = 0;
  for (int b = 31; b >= 0; --b) {
    const int c = temp[b];
    temp[32 + b] = s;
    s += c;
  }
}

__global__ void k_order_scatter(const int2* __restrict__ ranges, int n_items, int* __restrict__ temp,
                                int* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n_items;
  const int b = valid ? order_bucket(ranges, i) : -1;
  uint64_t remaining = __ballot(valid);
  while (remaining) {
    const int leader = __builtin_ctzll(remaining);
    const int lb = __shfl(b, leader, 64);
    const uint64_t same = __ballot(valid && b == lb);
    int base = 0;
    if (lane == leader) base = atomicAdd(&temp[32 + lb], __popcll(same));
    base = __shfl(base, leader, 64);
    if (valid && b == lb) {
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
      order[base + rank] = i;
    }
    remaining &= ~same;
  }
}

}  // namespace

void launch_render_fwd(const Raster& R, const FwdArgs& a, hipStream_t s) {
  if (a.stats) {
    hipLaunchKernelGGL(k_render_fwd<true>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
    hipLaunchKernelGGL(k_count_bwd_pairs, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  } else if (a.blocks > 0) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 0u, 1, s);
    hipLaunchKernelGGL(k_render_fwd_persistent, dim3((unsigned)a.blocks), dim3(kTileThreads), 0, s, R, a);
  } else {
    hipLaunchKernelGGL(k_render_fwd<false>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  }
}

void launch_render_bwd(const Raster& R, const BwdArgs& a, hipStream_t s) {
  const dim3 tb(kTileThreads);
  const bool det = a.part != nullptr;
  // ten fields: block walk; the six of a pose-only backward: quadrant walk
  if (a.blocks > 0) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 0u, 1, s);
    const dim3 grid((unsigned)a.blocks);
    if (a.geom_only) {
      if (det) hipLaunchKernelGGL(k_render_bwd_quad_persistent<true>, grid, tb, 0, s, R, a);
      else hipLaunchKernelGGL(k_render_bwd_quad_persistent<false>, grid, tb, 0, s, R, a);
    } else {
      if (det) hipLaunchKernelGGL(k_render_bwd_block_persistent<true>, grid, tb, 0, s, R, a);
      else hipLaunchKernelGGL(k_render_bwd_block_persistent<false>, grid, tb, 0, s, R, a);
    }
  } else {
    const dim3 grid((unsigned)a.n_items);
    if (a.geom_only) {
      if (det) hipLaunchKernelGGL(k_render_bwd_quad<true>, grid, tb, 0, s, R, a);
      else hipLaunchKernelGGL(k_render_bwd_quad<false>, grid, tb, 0, s, R, a);
    } else {
      if (det) hipLaunchKernelGGL(k_render_bwd_block<true>, grid, tb, 0, s, R, a);
      else hipLaunchKernelGGL(k_render_bwd_block<false>, grid, tb, 0, s, R, a);
    }
  }
}

void launch_det_rev(const Raster& R, const int2* ranges, const uint32_t* ids, const int4* rect, const uint32_t* goff,
                    uint32_t* rev, int n_items, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(k_det_rev, dim3((unsigned)n_items), dim3(256), 0, s, R, ranges, ids, rect, goff, rev);
}

void launch_det_reduce(const int4* rect, const uint32_t* goff, const uint32_t* rev, const uint32_t* mask,
                       const float* part, int64_t n_rec, bool geom_only, float* g2d, hipStream_t s) {
  if (n_rec <= 0) return;
  const int nf = geom_only ? 6 : 10;
  const unsigned g = (unsigned)((n_rec * nf + 255) / 256);
  if (geom_only)
    hipLaunchKernelGGL(k_det_reduce<6>, dim3(g), dim3(256), 0, s, rect, goff, rev, mask, part, n_rec, g2d);
  else
    hipLaunchKernelGGL(k_det_reduce<10>, dim3(g), dim3(256), 0, s, rect, goff, rev, mask, part, n_rec, g2d);
}

void launch_item_order(const int2* ranges, int n_items, int* order, int* temp, hipStream_t s) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(temp), 0u, 64, s);
  const unsigned g = (unsigned)((n_items + 255) / 256);
  hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, s, ranges, n_items, temp);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, temp);
  hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, s, ranges, n_items, temp, order);
}

}  // namespace gsr
