// kernels.hip -- the radar-scan hot path on CDNA4 (gfx950).
//
// Wavefront organisation:
//   k_raygen  primaries of every scan from the counter-based generator
//             (Sec. III-A, Eq. 2), appended to ray queue 0;
//   k_trace   (per bounce level) closest hit of every queued ray through the
//             BVH: persistent lanes that take a new ray as soon as theirs is
//             done (rays claimed 64 at a time from per-segment cursors), up
//             to kNodeSteps node steps between two scheduling decisions,
//             leaf tests batched wave-wide, and on levels with few rays per
//             lane idle lanes helping the wave's unfinished rays;
//   k_shade   (per bounce level) the interaction at each hit (Snell,
//             Fresnel, standard BRDF return, Sec. III-A), the return binned
//             into the polar image with a 64-bit fixed-point atomic
//             (Sec. III-B), and up to two children appended to the next queue
//             (one reservation per 512-lane block step);
//   k_scan    the optional one-launch form of k_trace + k_shade over every
//             level, each wave keeping its own rays' children.
//
// Floating-point rules: no contraction except where fmaf is written; the
// closest-hit, bin and total-internal-reflection decisions and the child
// geometry are float32 in a fixed order; energies are float64, except the
// specular lobe's power c^C, float32 in a form that keeps its relative
// accuracy near the specular direction (lobe_pow).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "philox.h"

#pragma clang fp contract(off)

namespace rr {

// Set bits of a wave-wide mask in the lanes below this one (the exclusive
// prefix count of a ballot): v_mbcnt_lo over lanes 0-31, v_mbcnt_hi over 32-63.
__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Claims this wave's next `pool` rays of a queue of n_in rays.  The queue is
// split into kCtrSegs segments, each with its own cursor (`cur`, one cursor
// per kCtrCursorStride words, so on its own cache line): one cursor
// serialised every wave's claims.  A wave starts at segment `seg` and moves
// on cyclically once that one is used up; `tries` counts the segments found
// used up.  On success the rays are [next, end); false once every segment is
// used up.  Wave-uniform; lane 0 does the atomics.
__device__ __forceinline__ bool claim_rays(uint32_t* cur, uint32_t n_in, uint32_t pool, uint32_t lane,
                                           uint32_t& seg, uint32_t& tries, uint32_t& next, uint32_t& end) {
#pragma unroll 1
  for (;;) {
    const uint32_t s0 = (uint32_t)((uint64_t)n_in * seg / kCtrSegs);
    const uint32_t s1 = (uint32_t)((uint64_t)n_in * (seg + 1u) / kCtrSegs);
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(cur + seg * kCtrCursorStride, pool);
    base = __shfl(base, 0);
    if (base < s1 - s0) {
      next = s0 + base;
      end = min(next + pool, s1);
      return true;
    }
    if (++tries >= kCtrSegs) return false;
    seg = (seg + 1u) & (kCtrSegs - 1u);
  }
}

constexpr uint32_t kHashBits = 11;     // shade: LDS table of 2048 accumulator cells
constexpr uint32_t kHashSlots = 1u << kHashBits;
constexpr uint32_t kHashEmpty = 0xffffffffu;

// Primary ray (k, i) of a scan: D3 cone offset (Eq. 2) around azimuth
// 2*pi*k/N_az, float64 then rounded to float32.
__device__ __forceinline__ void gen_primary(const DevScan& s, uint32_t k, uint32_t i, float& dx,
                                            float& dy, float& dz, float& g) {
  uint64_t ck = (s.flags & 2u) ? 0u : k;
  uint64_t ci = (s.flags & 4u) ? (uint64_t)(i >> 1) : (uint64_t)i;
  uint64_t x[4];
  philox4x64_10(s.seed, (uint64_t)s.scan_id, ck, ci, 0, 0, x);
  const double two53 = 1.0 / 9007199254740992.0;
  double u1 = (double)((x[0] >> 11) + 1u) * two53;
  double u2 = (double)(x[1] >> 11) * two53;
  double u3 = (double)(x[2] >> 11) * two53;
  double zz = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  double omega = -M_PI + 2.0 * M_PI * u3;
  double r = zz * s.sigma_r;
  double az_off = r * cos(omega), inc_off = r * sin(omega);
  // elliptic beam (Sec. III-A): the cone stretched along the two axes
  if (s.stretch_az != 1.0f) az_off = az_off * (double)s.stretch_az;
  if (s.stretch_inc != 1.0f) inc_off = inc_off * (double)s.stretch_inc;
  if ((s.flags & 4u) && (i & 1u)) az_off = -az_off;
  double phi = 2.0 * M_PI * (double)k / (double)s.n_az + az_off;
  double theta = inc_off;
  double ct = cos(theta);
  double ds0 = ct * cos(phi), ds1 = ct * sin(phi), ds2 = sin(theta);
  double w0 = s.R[0] * ds0 + s.R[1] * ds1 + s.R[2] * ds2;
  double w1 = s.R[3] * ds0 + s.R[4] * ds1 + s.R[5] * ds2;
  double w2 = s.R[6] * ds0 + s.R[7] * ds1 + s.R[8] * ds2;
  double len = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
  dx = (float)(w0 / len);
  dy = (float)(w1 / len);
  dz = (float)(w2 / len);
  g = (s.flags & 1u) ? (float)exp(-0.5 * zz * zz) : 1.0f;
}

// Unpolarised Fresnel reflectance from index N1 into N2 at incidence cosine
// ci (float64); 1 beyond the critical angle.
__device__ __forceinline__ double fresnel_unpolarised(double N1, double N2, double ci) {
  const double e = N1 / N2;
  const double k64 = 1.0 - e * e * (1.0 - ci * ci);
  if (k64 < 0.0) return 1.0;
  const double ct = sqrt(k64);
  const double ds = N1 * ci + N2 * ct, dp = N2 * ci + N1 * ct;
  if (ds == 0.0 || dp == 0.0) return 1.0;
  const double rs = (N1 * ci - N2 * ct) / ds;
  const double rp = (N2 * ci - N1 * ct) / dp;
  return 0.5 * (rs * rs + rp * rp);
}

// Share of the reflected energy a Cook-Torrance surface returns into the
// beam cone around unit direction v, for a ray of direction d meeting it
// with facing normal nf: f(l, v) (n.v) Omega with l = -d, clamped to [0, 1];
// f = k_d / pi + (1 - k_d) D F G1 G1 / (4 (n.l)(n.v)) with the GGX
// distribution, separable Smith masking and the unpolarised Fresnel factor
// (Walter et al., EGSR 2007).  Float64 in a fixed order.
__device__ __forceinline__ double ct_return(const DevMaterial& M, float nfx, float nfy, float nfz, float dx,
                                            float dy, float dz, float vx, float vy, float vz) {
  const double n0 = nfx, n1 = nfy, n2 = nfz;
  const double l0 = -(double)dx, l1 = -(double)dy, l2 = -(double)dz;
  const double v0 = vx, v1 = vy, v2 = vz;
  const double nl = n0 * l0 + n1 * l1 + n2 * l2;
  const double nv = n0 * v0 + n1 * v1 + n2 * v2;
  double f = 0.0;
  if (nl > 0.0 && nv > 0.0) {
    double h0 = l0 + v0, h1 = l1 + v1, h2 = l2 + v2;
    const double hl = sqrt(h0 * h0 + h1 * h1 + h2 * h2);
    h0 = h0 / hl;
    h1 = h1 / hl;
    h2 = h2 / hl;
    const double nh = n0 * h0 + n1 * h1 + n2 * h2;
    const double vh = v0 * h0 + v1 * h1 + v2 * h2;
    const double a = M.beta, a2 = a * a;
    const double q = nh * nh * (a2 - 1.0) + 1.0;
    const double D = a2 / (M_PI * q * q);
    const double g1l = 2.0 * nl / (nl + sqrt(a2 + (1.0 - a2) * nl * nl));
    const double g1v = 2.0 * nv / (nv + sqrt(a2 + (1.0 - a2) * nv * nv));
    const double F = fresnel_unpolarised(1.0, (double)M.n, vh);
    const double kd = M.a;
    f = kd / M_PI + (1.0 - kd) * D * F * g1l * g1v / (4.0 * nl * nv);
  }
  const double w = f * nv * M.s;
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}

// c^C of the specular lobe of the standard BRDF (Eq. 5) for c in [0, 1],
// given u = c - 1 (-1 <= u <= 0) in float32: c^C = exp(C log1p(u)).  With
// the lobe's large exponents (C up to a few thousand) c^C is only
// non-negligible for c within ~1e-2 of 1, where rounding c itself would
// cost C ulps of relative accuracy; u keeps its own relative accuracy there.
// u <= -1 means c <= 0: the lobe is 0 (1 for C = 0, as pow(0, 0)).
__device__ __forceinline__ float lobe_pow(float u, float C) {
  if (u <= -1.0f) return C == 0.0f ? 1.0f : 0.0f;
  return expf(C * log1pf(u));
}

// Origin offset of Waechter & Binder (Ray Tracing Gems, 2019, ch. 6).
__device__ __forceinline__ float offset1(float p, float n) {
  const float origin = 1.0f / 32.0f, float_scale = 1.0f / 65536.0f, int_scale = 256.0f;
  int of = (int)(int_scale * n);
  float pi = __int_as_float(__float_as_int(p) + ((p < 0.0f) ? -of : of));
  return fabsf(p) < origin ? p + float_scale * n : pi;
}

__device__ __forceinline__ void normalize3(float& x, float& y, float& z) {
  float len = sqrtf(dot3(x, y, z, x, y, z));
  x = x / len;
  y = y / len;
  z = z / len;
}

// Closest-hit traversal, persistent and replenishing (after Aila & Laine,
// "Understanding the efficiency of ray traversal on GPUs", HPG 2009): every
// lane owns one ray at a time; lanes whose ray has finished take new rays
// (claim_rays, one atomic per wave and claim) as soon as A.refill lanes are
// idle.
//
// Each loop iteration is either a node step or a triangle phase, decided for
// the whole wave.  In a node step every tracing lane visits one inner node:
// inner children hit by the ray go nearest-first onto its stack (LDS, entry s
// of lane t at stk[s * B], entries beyond kStack in the workspace), hit leaf
// children are appended to the wave's leaf ring in LDS.  A triangle phase
// takes up to 64 ring entries, one per lane, and tests the leaf's triangles
// for the ray of the lane that appended it; hits meet in a per-lane LDS word
// holding min over (t, original triangle id), updated with a 64-bit LDS
// atomic min.  The closest hit is that minimum whatever the order of the
// tests, and a box is culled only beyond the current minimum, so batching
// leaves changes speed, never the result.  A lane finishes its ray once its
// stack is empty and the ring has passed its last entry.
//
// kShadow: the same traversal for the air-path visibility rays of the level,
// each bounded by its distance to the sensor (a triangle at 0 < t <= dist
// blocks it).  A ray stops walking at its first blocker, and an unblocked
// return is added to the image accumulator.
//
// kHelp: tail helping, for levels with few rays per lane, whose time is the
// walk of their longest rays.  Once a wave has no rays left to claim, its
// idle lanes take the bottom entry (the oldest, usually the largest subtree)
// of a walking lane's stack and walk that subtree for the same ray: the
// leaves they queue carry the owner's lane, so their hits meet in the
// owner's (t, id) minimum, and they cull against that minimum.  The owner
// finishes once no helper walks for it.  The result is the same minimum, so
// images and records do not change.  Held to 80 registers, as the plain
// variant, so that both keep 24 waves per CU resident.
template <bool kCount, bool kShadow, bool kHelp>
__global__ void __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(kHelp ? 6 : 1)))
k_trace(LevelArgs A) {
  __shared__ int32_t lds_stack[kStack * kTraceBlock];
  __shared__ uint32_t lds_leaf[kTraceBlock / 64][kLeafRing];     // leaf reference
  __shared__ uint8_t lds_own[kTraceBlock / 64][kLeafRing];       // lane that appended it
  __shared__ unsigned long long lds_best[kTraceBlock];           // (t bits << 32) | original id
  __shared__ uint32_t lds_help[kHelp ? kTraceBlock : 1];          // helpers walking for each lane's ray
  __shared__ uint8_t lds_pair[kHelp ? kTraceBlock / 64 : 1][64];  // victim lane of each helper rank
  int32_t* stk = lds_stack + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = threadIdx.x >> 6;
  const uint32_t wave_base = threadIdx.x - lane;
  const uint32_t n_in = kShadow ? min(A.counters[kCtrShadow], A.shq_cap) : min(A.counters[kCtrCount + A.depth], A.cap);
  const Node4* __restrict__ nodes = A.nodes;
  const float4* __restrict__ tris = A.tris;
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t spill_stride = gridDim.x * blockDim.x;
  const uint32_t tri_batch = min(max(A.tri_batch, 1u), 64u);

  bool valid = false, exhausted = false;
  uint32_t pool_next = 0, pool_end = 0;  // wave-uniform: claimed, not yet started rays
  // rays are claimed from segment cursors (claim_rays), starting at the
  // block's segment; closest-hit levels use cursor set `depth`, the
  // visibility launch the set after the last level's
  uint32_t seg = blockIdx.x & (kCtrSegs - 1u), seg_tries = 0;
  uint32_t* const seg_cur =
      A.counters + kCtrCursor + (kShadow ? kMaxLevels : A.depth) * kCtrSegs * kCtrCursorStride;
  uint32_t ring_head = 0, ring_tail = 0;  // wave-uniform: appended / tested ring entries
  uint32_t ridx = 0, visits = 0, excl = 0xffffffffu, last_pos = 0;
  float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, best_t = 0;
  RayBox rb{};
  int32_t cur = 0;
  int sp = 0;
  bool trav_done = false;  // stack empty (or visit bound reached)
  uint32_t cnt_nodes = 0, cnt_tris = 0, cnt_rays = 0;
  uint64_t cnt_iters = 0, cnt_active = 0, cnt_tail_iters = 0, cnt_tail_active = 0;  // wave-uniform
  uint32_t cnt_max_visits = 0;
  // tail helping: the lane whose ray this lane walks (itself unless it is a
  // helper), the stack entries below sb handed to helpers
  uint32_t owner = lane;
  int sb = 0;
  bool helper = false;
  uint32_t guard = 0;
  if (kHelp) lds_help[threadIdx.x] = 0u;

  for (;;) {
    // a bound every wave reaches: a level takes far fewer iterations per
    // wave than this (tens of thousands at the largest sizes); should the
    // helpers' bookkeeping ever fail to drain, the launch still ends and the
    // scan reports it
    if (kHelp && ++guard > (1u << 22)) {
      if (lane == 0) atomicOr(A.counters + kCtrOverflow, kOverflowSteps);
      break;
    }
    // ---- refill idle lanes (wave-uniform decision) from the wave's pool of
    // claimed rays; the pool is refilled A.pool rays at a time with one atomic
    // on a segment cursor
    uint64_t idle = __ballot(!valid);
    if (!exhausted && (uint32_t)__popcll(idle) >= A.refill) {
#pragma unroll 1
      for (int pass = 0; pass < 2 && idle; ++pass) {
        if (pool_next >= pool_end &&
            !claim_rays(seg_cur, n_in, A.pool, lane, seg, seg_tries, pool_next, pool_end)) {
          exhausted = true;
          break;
        }
        const uint32_t take = min((uint32_t)__popcll(idle), pool_end - pool_next);
        const uint32_t rank = lane_prefix(idle);
        const bool mine = !valid && rank < take;
        if (mine) {
          const uint32_t my = pool_next + rank;
          float4 a, b;
          if constexpr (kShadow) {
            a = A.shq.a[my];
            b = A.shq.b[my];
            excl = A.shq.c[my].w;
            best_t = a.w;
          } else {
            a = A.in.a[my];
            b = A.in.b[my];
            const uint32_t m = A.in.m[my];
            excl = A.in.c[my].w;
            const uint32_t medium = (m >> 8) & 0xffu;
            const float n_cur = medium == kAir ? 1.0f : A.mats[medium].n;
            best_t = (A.scans[m >> 16].r_max - a.w) / n_cur;
          }
          lds_best[threadIdx.x] = ((unsigned long long)__float_as_uint(best_t) << 32) | 0xffffffffull;
          ox = a.x;
          oy = a.y;
          oz = a.z;
          dx = b.x;
          dy = b.y;
          dz = b.z;
          ray_box_setup(ox, oy, oz, dx, dy, dz, rb);
          ridx = my;
          cur = 0;
          sp = 0;
          sb = 0;
          owner = lane;
          helper = false;
          visits = 0;
          last_pos = ring_head;
          trav_done = false;
          valid = true;
          if (kCount) ++cnt_rays;
        }
        pool_next += take;
        idle = __ballot(!valid);
      }
    }
    const uint64_t live = __ballot(valid);
    if (live == 0ull) break;  // only once the level is exhausted
    if (kCount) {
      ++cnt_iters;
      cnt_active += (uint64_t)__popcll(live);
      if (exhausted) {
        ++cnt_tail_iters;
        cnt_tail_active += (uint64_t)__popcll(live);
      }
    }

    // ---- node step or triangle phase.  A node step may append up to four
    // leaves per lane, so it runs only while the ring has room for that.
    const uint64_t walking = __ballot(valid && !trav_done);
    const uint32_t queued = ring_head - ring_tail;
    const bool tri_phase = queued >= tri_batch ||
                           (queued > 0 && (walking == 0ull || queued + 4u * (uint32_t)__popcll(walking) > kLeafRing));
    if (tri_phase) {
      const uint32_t n = min(queued, 64u);
      const bool take = lane < n;
      const uint32_t pos = (ring_tail + lane) & (kLeafRing - 1u);
      const uint32_t ref = take ? lds_leaf[wib][pos] : 0u;
      const int own = take ? (int)lds_own[wib][pos] : (int)lane;
      const float rox = __shfl(ox, own), roy = __shfl(oy, own), roz = __shfl(oz, own);
      const float rdx = __shfl(dx, own), rdy = __shfl(dy, own), rdz = __shfl(dz, own);
      const uint32_t rexcl = __shfl(excl, own);
      if (take) {
        unsigned long long cb = lds_best[wave_base + own];
        float tmax = __uint_as_float((uint32_t)(cb >> 32));
        const uint32_t start = leaf_start((int32_t)ref), count = leaf_count((int32_t)ref);
#pragma unroll 1
        for (uint32_t k = 0; k < count; ++k) {
          const uint32_t li = start + k;
          const float4 ta = tris[3 * li + 0];
          const uint32_t orig = __float_as_uint(ta.w);
          if (orig == rexcl) continue;
          if (kCount) ++cnt_tris;
          const float4 e1 = tris[3 * li + 1];
          const float4 e2 = tris[3 * li + 2];
          float t;
          if (ray_tri(rox, roy, roz, rdx, rdy, rdz, ta.x, ta.y, ta.z, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z,
                      tmax, t)) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | orig;
            if (key < cb) {
              atomicMin(&lds_best[wave_base + own], key);
              cb = key;
              tmax = t;
            }
          }
        }
      }
      ring_tail += n;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        const unsigned long long mine = lds_best[wave_base + (kHelp ? owner : lane)];
        best_t = __uint_as_float((uint32_t)(mine >> 32));
        // a visibility ray is done at its first blocker
        if (kShadow && (uint32_t)mine != 0xffffffffu) trav_done = true;
      }
    } else {
      // up to kNodeSteps node steps in a row, each only while the ring has
      // room for four more leaves per walking lane; the refill, triangle and
      // completion checks run once per run of steps
#pragma unroll 1
      for (uint32_t step = 0;;) {
        // Every lane runs the node step; one without a node to visit (idle,
        // done, or holding a reference outside the tree) reads the root and
        // pushes and appends nothing.  Predication instead of a branch keeps
        // the per-child conditions as wave masks.
        const bool walk = valid && !trav_done;
        // top of the LDS stack, read ahead of the decision to pop so the pop
        // stays an LDS access (entries beyond kStack come from the workspace)
        const int32_t top = stk[min(max(sp - 1, 0), kStack - 1) * kTraceBlock];
        // a reference outside the tree (kEmpty: none) takes the next stack
        // entry; a popped entry still outside it is dropped at the next step
        if (walk && (uint32_t)cur >= A.n_nodes) {
          if (sp > sb) {
            --sp;
            cur = sp < kStack ? top : A.spill[(size_t)(sp - kStack) * spill_stride + gtid];
          } else {
            trav_done = true;
          }
        }
        const bool vis = walk & !trav_done & ((uint32_t)cur < A.n_nodes);
        const float4* np = reinterpret_cast<const float4*>(nodes + (vis ? cur : 0));
        const float4 w0 = np[0];
        const uint4 w1 = reinterpret_cast<const uint4*>(np)[1];
        const uint4 w2 = reinterpret_cast<const uint4*>(np)[2];
        const int4 w3 = reinterpret_cast<const int4*>(np)[3];
        if (kCount && vis) ++cnt_nodes;
        float tn[4];
        bool hit[4];
        node4_slabs(w0, w1, w2, rb, best_t, tn, hit);
        const int32_t lref[4] = {w3.x, w3.y, w3.z, w3.w};
        // hit inner children far to near, everything else last: 5 compare-exchanges
        bool lf[4];
        float key[4];
        int32_t val[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // bitwise, not short-circuit: no branches around the conditions
          const bool inner = vis & hit[j] & (lref[j] >= 0);
          lf[j] = vis & hit[j] & (lref[j] < 0);
          key[j] = inner ? tn[j] : -INFINITY;
          val[j] = inner ? lref[j] : kEmpty;
        }
#define RR_CX(i, j)                     \
  if (key[j] > key[i]) {                \
    const float tk = key[i];            \
    key[i] = key[j];                    \
    key[j] = tk;                        \
    const int32_t tv = val[i];          \
    val[i] = val[j];                    \
    val[j] = tv;                        \
  }
        RR_CX(0, 1) RR_CX(2, 3) RR_CX(0, 2) RR_CX(1, 3) RR_CX(1, 2)
#undef RR_CX
        // h hit inner children sit in entries 0 .. h - 1; the nearest, entry
        // h - 1, is visited next and the h - 1 others are pushed farthest
        // first.  Where three slots are free in LDS all three are written
        // unconditionally (slots at or above the new top are unused, and a
        // lane that visits nothing pushes nothing); otherwise entry by entry,
        // deeper ones into the workspace.  The builder bounds the worst-case
        // depth by kStack + kSpill.
        const bool m1 = key[1] > -INFINITY, m2 = key[2] > -INFINITY, m3 = key[3] > -INFINITY;
        const int pushes = (int)m1 + (int)m2 + (int)m3;
        if (sp + 3 <= kStack) {
          stk[(sp + 0) * kTraceBlock] = val[0];
          stk[(sp + 1) * kTraceBlock] = val[1];
          stk[(sp + 2) * kTraceBlock] = val[2];
          sp += pushes;
        } else {
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            if (j < pushes && sp < kStack + kSpill) {
              if (sp < kStack)
                stk[sp * kTraceBlock] = val[j];
              else
                A.spill[(size_t)(sp - kStack) * spill_stride + gtid] = val[j];
              ++sp;
            }
          }
        }
        if (vis) {
          cur = m3 ? val[3] : m2 ? val[2] : m1 ? val[1] : val[0];
          // every node is entered at most once per ray; the bound only guards
          // against a malformed tree
          if (++visits > A.n_nodes) trav_done = true;
        }
        // hit leaves into the ring, slot by slot: the lanes with a leaf in slot
        // j take consecutive entries (one ballot and one prefix count per
        // slot).  All lanes take part, so the ring head stays the same in
        // every lane; a lane's leaves all lie before the step's final head.
        const uint64_t l0 = __ballot(lf[0]), l1 = __ballot(lf[1]);
        const uint64_t l2 = __ballot(lf[2]), l3 = __ballot(lf[3]);
        if (l0 | l1 | l2 | l3) {
          uint32_t p = ring_head;
          const uint64_t lm[4] = {l0, l1, l2, l3};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (lm[j]) {
              if (lf[j]) {
                const uint32_t pos = (p + lane_prefix(lm[j])) & (kLeafRing - 1u);
                lds_leaf[wib][pos] = (uint32_t)lref[j];
                lds_own[wib][pos] = (uint8_t)(kHelp ? owner : lane);
              }
              p += (uint32_t)__popcll(lm[j]);
            }
          }
          if (lf[0] || lf[1] || lf[2] || lf[3]) last_pos = p;
          ring_head = p;
        }
        if (++step >= kNodeSteps) break;
        const uint64_t still = __ballot(valid && !trav_done);
        if (still == 0ull || ring_head - ring_tail + 4u * (uint32_t)__popcll(still) > kLeafRing) break;
      }
    }
    __builtin_amdgcn_wave_barrier();

    // ---- rays whose traversal and leaf tests are complete; a helper is done
    // with its subtree, an owner waits until no helper walks for its ray
    if (kHelp && helper && valid && trav_done && (int32_t)(ring_tail - last_pos) >= 0) {
      atomicSub(&lds_help[wave_base + owner], 1u);
      valid = false;
      helper = false;
    }
    __builtin_amdgcn_wave_barrier();
    if (valid && trav_done && (int32_t)(ring_tail - last_pos) >= 0 &&
        (!kHelp || lds_help[threadIdx.x] == 0u)) {
      if (kCount) cnt_max_visits = max(cnt_max_visits, visits);
      const unsigned long long b = lds_best[threadIdx.x];
      if constexpr (kShadow) {
        const bool blocked = (uint32_t)b != 0xffffffffu;
        if (!blocked) {
          const uint4 c = A.shq.c[ridx];
          const unsigned long long qv = ((unsigned long long)c.y << 32) | c.x;
          if (qv) atomicAdd(A.acc + c.z, qv);
        }
        if (A.air_rec) {
          const uint32_t slot = __float_as_uint(A.shq.b[ridx].w);
          if (slot != 0xffffffffu) A.air_rec[slot] = blocked ? 1 : 0;
        }
      } else {
        A.hits[ridx] = make_uint2((uint32_t)(b >> 32), (uint32_t)b);
      }
      valid = false;
    }

    // ---- tail helping: once no rays are left to claim, idle lanes take the
    // bottom entry of a walking lane's stack (two or more entries, all in
    // LDS) and walk that subtree for the same ray; leaves they queue carry
    // the owner's lane, so their hits meet in the owner's minimum
    if (kHelp && exhausted) {
      __builtin_amdgcn_wave_barrier();
      const bool can_give = valid && !trav_done && sp - sb >= 2 && sp <= kStack;
      const uint64_t idle_m = __ballot(!valid);
      const uint64_t give_m = __ballot(can_give);
      const uint32_t k = min((uint32_t)__popcll(idle_m), (uint32_t)__popcll(give_m));
      if (k) {
        const uint32_t rv = lane_prefix(give_m), ri = lane_prefix(idle_m);
        const bool victim = can_give && rv < k;
        if (victim) lds_pair[wib][rv] = (uint8_t)lane;
        __builtin_amdgcn_wave_barrier();
        const bool takes = !valid && ri < k;
        const int v = takes ? (int)lds_pair[wib][ri] : (int)lane;
        const int vsb = __shfl(sb, v);
        const uint32_t vown = (uint32_t)__shfl((int)owner, v);
        const float rox = __shfl(ox, v), roy = __shfl(oy, v), roz = __shfl(oz, v);
        const float rdx = __shfl(dx, v), rdy = __shfl(dy, v), rdz = __shfl(dz, v);
        const uint32_t rexcl = (uint32_t)__shfl((int)excl, v);
        if (takes) {
          cur = lds_stack[vsb * kTraceBlock + wave_base + (uint32_t)v];
          owner = vown;
          ox = rox;
          oy = roy;
          oz = roz;
          dx = rdx;
          dy = rdy;
          dz = rdz;
          excl = rexcl;
          ray_box_setup(ox, oy, oz, dx, dy, dz, rb);
          best_t = __uint_as_float((uint32_t)(lds_best[wave_base + vown] >> 32));
          atomicAdd(&lds_help[wave_base + vown], 1u);
          sp = 0;
          sb = 0;
          visits = 0;
          last_pos = ring_head;
          trav_done = false;
          valid = true;
          helper = true;
        }
        if (victim) ++sb;
      }
    }
  }
  if (kCount) {
    atomicAdd(A.prof + 0, (unsigned long long)cnt_nodes);
    atomicAdd(A.prof + 1, (unsigned long long)cnt_tris);
    atomicAdd(A.prof + 2, (unsigned long long)cnt_rays);
    atomicMax(A.prof + kProfMaxVisits + A.depth, (unsigned long long)cnt_max_visits);
    if (lane == 0) {
      atomicAdd(A.prof + kProfIters + A.depth, (unsigned long long)cnt_iters);
      atomicAdd(A.prof + kProfActive + A.depth, (unsigned long long)cnt_active);
      atomicAdd(A.prof + kProfTailIters + A.depth, (unsigned long long)cnt_tail_iters);
      atomicAdd(A.prof + kProfTailActive + A.depth, (unsigned long long)cnt_tail_active);
    }
  }
}

// Closest-hit traversal of the eight-wide tree (after Ylitie, Karras and
// Laine, "Efficient incoherent ray traversal on GPUs through compressed wide
// BVHs", HPG 2017): instead of sorting hit children, a node's hit inner
// children form a group (first child, hit slots in the ray's octant order,
// inner-slot mask) and the traversal takes them lowest order bit first; a
// visit pushes at most the rest of the current group.  Hit leaves go to the
// wave's leaf ring (one 32-bit entry: lane << 26 | (count - 1) << 24 | first
// triangle) and are tested in triangle phases exactly as in k_trace; the
// refill, the per-lane (t, original id) minimum and the completion rule are
// those of k_trace.
template <bool kCount>
__global__ void __launch_bounds__(kTraceBlock) k_trace8(LevelArgs A) {
  __shared__ uint2 lds_gstack[kStack8 * kTraceBlock];           // node groups
  __shared__ uint32_t lds_leaf[kTraceBlock / 64][kLeafRing8];
  __shared__ unsigned long long lds_best[kTraceBlock];
  uint2* gstk = lds_gstack + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = threadIdx.x >> 6;
  const uint32_t wave_base = threadIdx.x - lane;
  const uint32_t n_in = min(A.counters[kCtrCount + A.depth], A.cap);
  uint32_t seg = blockIdx.x & (kCtrSegs - 1u), seg_tries = 0;  // claim_rays state
  uint32_t* const seg_cur = A.counters + kCtrCursor + A.depth * kCtrSegs * kCtrCursorStride;
  const Node8* __restrict__ nodes = A.nodes8;
  const float4* __restrict__ tris = A.tris;
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t spill_stride = gridDim.x * blockDim.x;
  uint2* const spill = reinterpret_cast<uint2*>(A.spill);
  const uint32_t tri_batch = min(max(A.tri_batch, 1u), 64u);

  bool valid = false, exhausted = false;
  uint32_t pool_next = 0, pool_end = 0;
  uint32_t ring_head = 0, ring_tail = 0;
  uint32_t ridx = 0, visits = 0, excl = 0xffffffffu, last_pos = 0, oct = 0;
  float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, best_t = 0;
  RayBox rb{};
  int32_t cur = 0;                     // node to visit (-1: take one from the group)
  uint32_t g_base = 0, g_mask = 0;     // current group
  int sp = 0;
  bool trav_done = false;
  uint32_t cnt_nodes = 0, cnt_tris = 0, cnt_rays = 0;
  uint64_t cnt_iters = 0, cnt_active = 0, cnt_tail_iters = 0, cnt_tail_active = 0;
  uint32_t cnt_max_visits = 0;

  for (;;) {
    uint64_t idle = __ballot(!valid);
    if (!exhausted && (uint32_t)__popcll(idle) >= A.refill) {
#pragma unroll 1
      for (int pass = 0; pass < 2 && idle; ++pass) {
        if (pool_next >= pool_end &&
            !claim_rays(seg_cur, n_in, A.pool, lane, seg, seg_tries, pool_next, pool_end)) {
          exhausted = true;
          break;
        }
        const uint32_t take = min((uint32_t)__popcll(idle), pool_end - pool_next);
        const uint32_t rank = lane_prefix(idle);
        if (!valid && rank < take) {
          const uint32_t my = pool_next + rank;
          const float4 a = A.in.a[my];
          const float4 b = A.in.b[my];
          const uint32_t m = A.in.m[my];
          excl = A.in.c[my].w;
          const uint32_t medium = (m >> 8) & 0xffu;
          const float n_cur = medium == kAir ? 1.0f : A.mats[medium].n;
          best_t = (A.scans[m >> 16].r_max - a.w) / n_cur;
          lds_best[threadIdx.x] = ((unsigned long long)__float_as_uint(best_t) << 32) | 0xffffffffull;
          ox = a.x;
          oy = a.y;
          oz = a.z;
          dx = b.x;
          dy = b.y;
          dz = b.z;
          ray_box_setup(ox, oy, oz, dx, dy, dz, rb);
          oct = ray_octant(rb);
          ridx = my;
          cur = 0;
          g_mask = 0;
          sp = 0;
          visits = 0;
          last_pos = ring_head;
          trav_done = false;
          valid = true;
          if (kCount) ++cnt_rays;
        }
        pool_next += take;
        idle = __ballot(!valid);
      }
    }
    const uint64_t live = __ballot(valid);
    if (live == 0ull) break;
    if (kCount) {
      ++cnt_iters;
      cnt_active += (uint64_t)__popcll(live);
      if (exhausted) {
        ++cnt_tail_iters;
        cnt_tail_active += (uint64_t)__popcll(live);
      }
    }

    const uint64_t walking = __ballot(valid && !trav_done);
    const uint32_t queued = ring_head - ring_tail;
    const bool tri_phase = queued >= tri_batch ||
                           (queued > 0 && (walking == 0ull || queued + 8u * (uint32_t)__popcll(walking) > kLeafRing8));
    if (tri_phase) {
      const uint32_t n = min(queued, 64u);
      const bool take = lane < n;
      const uint32_t e = take ? lds_leaf[wib][(ring_tail + lane) & (kLeafRing8 - 1u)] : (lane << 26);
      const int own = (int)(e >> 26);
      const float rox = __shfl(ox, own), roy = __shfl(oy, own), roz = __shfl(oz, own);
      const float rdx = __shfl(dx, own), rdy = __shfl(dy, own), rdz = __shfl(dz, own);
      const uint32_t rexcl = __shfl(excl, own);
      if (take) {
        unsigned long long cb = lds_best[wave_base + own];
        float tmax = __uint_as_float((uint32_t)(cb >> 32));
        const uint32_t start = e & 0xffffffu, count = ((e >> 24) & 3u) + 1u;
#pragma unroll 1
        for (uint32_t k = 0; k < count; ++k) {
          const uint32_t li = start + k;
          const float4 ta = tris[3 * li + 0];
          const uint32_t orig = __float_as_uint(ta.w);
          if (orig == rexcl) continue;
          if (kCount) ++cnt_tris;
          const float4 e1 = tris[3 * li + 1];
          const float4 e2 = tris[3 * li + 2];
          float t;
          if (ray_tri(rox, roy, roz, rdx, rdy, rdz, ta.x, ta.y, ta.z, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z,
                      tmax, t)) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | orig;
            if (key < cb) {
              atomicMin(&lds_best[wave_base + own], key);
              cb = key;
              tmax = t;
            }
          }
        }
      }
      ring_tail += n;
      __builtin_amdgcn_wave_barrier();
      if (valid) best_t = __uint_as_float((uint32_t)(lds_best[threadIdx.x] >> 32));
    } else {
      uint32_t leaves = 0, l_first = 0, l_meta0 = 0, l_meta1 = 0;  // hit leaf slots of this visit
      if (valid && !trav_done) {
        if (cur < 0) {
          if ((g_mask & 0xffu) == 0u) {
            if (sp > 0) {
              --sp;
              const uint2 ge = sp < kStack8 ? gstk[sp * kTraceBlock]
                                            : spill[(size_t)(sp - kStack8) * spill_stride + gtid];
              g_base = ge.x;
              g_mask = ge.y;
            } else {
              trav_done = true;
            }
          }
          if (!trav_done) {
            const uint32_t i = (uint32_t)__builtin_ctz(g_mask & 0xffu);
            g_mask &= ~(1u << i);
            const uint32_t s = i ^ oct;
            cur = (int32_t)(g_base + (uint32_t)__popc((g_mask >> 8) & ((1u << s) - 1u)));
          }
        }
        if (!trav_done) {
          const float4* np = reinterpret_cast<const float4*>(nodes + cur);
          Node8 nd;
          nd.w0 = np[0];
          nd.w1 = reinterpret_cast<const uint4*>(np)[1];
          nd.w2 = reinterpret_cast<const uint4*>(np)[2];
          nd.w3 = reinterpret_cast<const uint4*>(np)[3];
          nd.w4 = reinterpret_cast<const uint4*>(np)[4];
          if (kCount) ++cnt_nodes;
          const uint32_t hits = node8_boxes(nd, rb, best_t);
          const uint32_t im = __float_as_uint(nd.w0.w) >> 24;
          leaves = hits & (nd.w1.y >> 24);
          l_first = nd.w1.y & 0xffffffu;
          l_meta0 = nd.w1.z;
          l_meta1 = nd.w1.w;
          const uint32_t inner = hits & im;
          if (inner) {
            if ((g_mask & 0xffu) && sp < kStack8 + kSpill / 2) {
              if (sp < kStack8)
                gstk[sp * kTraceBlock] = make_uint2(g_base, g_mask);
              else
                spill[(size_t)(sp - kStack8) * spill_stride + gtid] = make_uint2(g_base, g_mask);
              ++sp;
            }
            g_base = nd.w1.x;
            g_mask = octant_order(inner, oct) | (im << 8);
          }
          cur = -1;
          // every node is entered at most once per ray; the bound only guards
          // against a malformed tree
          if (++visits > A.n_nodes) trav_done = true;
        }
      }
      // hit leaves into the ring: exclusive prefix of the per-lane counts
      // from one ballot per count bit (all lanes take part)
      const uint32_t cnt = (uint32_t)__popc(leaves);
      uint32_t prefix = 0, total = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint64_t m = __ballot((cnt >> b) & 1u);
        prefix += lane_prefix(m) << b;
        total += (uint32_t)__popcll(m) << b;
      }
      uint32_t p = ring_head + prefix;
      while (leaves) {
        const uint32_t s = (uint32_t)__builtin_ctz(leaves);
        leaves &= leaves - 1u;
        const uint32_t meta = ((s < 4 ? l_meta0 : l_meta1) >> (8 * (s & 3u))) & 0xffu;
        lds_leaf[wib][p & (kLeafRing8 - 1u)] = (lane << 26) | ((meta >> 5) << 24) | (l_first + (meta & 31u));
        last_pos = ++p;
      }
      ring_head += total;
    }
    __builtin_amdgcn_wave_barrier();

    if (valid && trav_done && (int32_t)(ring_tail - last_pos) >= 0) {
      if (kCount) cnt_max_visits = max(cnt_max_visits, visits);
      const unsigned long long b = lds_best[threadIdx.x];
      A.hits[ridx] = make_uint2((uint32_t)(b >> 32), (uint32_t)b);
      valid = false;
    }
  }
  if (kCount) {
    atomicAdd(A.prof + 0, (unsigned long long)cnt_nodes);
    atomicAdd(A.prof + 1, (unsigned long long)cnt_tris);
    atomicAdd(A.prof + 2, (unsigned long long)cnt_rays);
    atomicMax(A.prof + kProfMaxVisits + A.depth, (unsigned long long)cnt_max_visits);
    if (lane == 0) {
      atomicAdd(A.prof + kProfIters + A.depth, (unsigned long long)cnt_iters);
      atomicAdd(A.prof + kProfActive + A.depth, (unsigned long long)cnt_active);
      atomicAdd(A.prof + kProfTailIters + A.depth, (unsigned long long)cnt_tail_iters);
      atomicAdd(A.prof + kProfTailActive + A.depth, (unsigned long long)cnt_tail_active);
    }
  }
}

// Wave-aggregated append of up to one ray per lane into a queue: one atomic
// per wave.  Returns the slot of this lane (valid only if `want`).
__device__ __forceinline__ uint32_t wave_append(bool want, uint32_t* counter, uint32_t lane,
                                                uint64_t& mask) {
  mask = __ballot(want);
  const uint32_t total = (uint32_t)__popcll(mask);
  uint32_t base = 0;
  if (total) {
    if (lane == 0) base = atomicAdd(counter, total);
    base = __shfl(base, 0);
  }
  return base + lane_prefix(mask);
}

__device__ __forceinline__ void put_ray(const QueueView& q, uint32_t slot, float ox, float oy, float oz,
                                        float L, float dx, float dy, float dz, float g, double E,
                                        uint32_t pid, uint32_t excl, uint32_t meta) {
  q.a[slot] = make_float4(ox, oy, oz, L);
  q.b[slot] = make_float4(dx, dy, dz, g);
  q.c[slot] = make_uint4((uint32_t)__double2loint(E), (uint32_t)__double2hiint(E), pid, excl);
  q.m[slot] = meta;
}

// Primary rays of every scan (level 0).  Work items are global primary
// indices; masked primaries are skipped; the rest are appended to queue 0.
__global__ void __launch_bounds__(kBlock) k_raygen(LevelArgs A) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t base = wave * 64u; base < A.n_first; base += n_waves * 64u) {
    const uint32_t gp = base + lane;
    bool active = gp < A.n_first;
    uint32_t scan = 0, pid = 0;
    float dx = 1, dy = 0, dz = 0, g = 1, ox = 0, oy = 0, oz = 0;
    double E = 0.0;
    if (active) {
      uint32_t lo = 0, hi = A.n_scans - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (A.scans[mid].prim_base <= gp)
          lo = mid;
        else
          hi = mid - 1;
      }
      scan = lo;
      const DevScan& s = A.scans[scan];
      pid = gp - s.prim_base;
      if (s.mask && !s.mask[pid]) {
        active = false;
      } else {
        const uint32_t k = pid / s.n_s, i = pid - k * s.n_s;
        gen_primary(s, k, i, dx, dy, dz, g);
        ox = s.pos[0];
        oy = s.pos[1];
        oz = s.pos[2];
        E = (double)s.e0;
      }
    }
    uint32_t slot = gp;  // no mask: primary gp sits at slot gp (count preset)
    if (A.masked) {
      uint64_t mask;
      slot = wave_append(active, A.counters + kCtrCount, lane, mask);
    }
    if (active && slot < A.cap)
      put_ray(A.out, slot, ox, oy, oz, 0.0f, dx, dy, dz, g, E, pid, 0xffffffffu,
              (scan << 16) | (kAir << 8) | 1u);
    else if (active)
      atomicOr(A.counters + kCtrOverflow, 1u);
  }
}

// ---------------------------------------------------------------- interaction
// What the interaction at one hit produces (Sec. III-A): the return to bin
// and up to two children.
struct Shaded {
  bool has_q = false, has_r = false, has_t = false;
  uint32_t cell = 0;              // accumulator cell of the return
  unsigned long long qv = 0;      // its fixed-point energy
  float range = 0.0f, g = 1.0f;   // one-way optical path at the hit; receive gain
  float rox = 0, roy = 0, roz = 0, rdx = 0, rdy = 0, rdz = 0;  // reflected child
  float tox = 0, toy = 0, toz = 0, tdx = 0, tdy = 0, tdz = 0;  // refracted child
  double e_refl = 0.0, e_refr = 0.0;
  uint32_t pid = 0, r_meta = 0, t_meta = 0;
  int32_t hit = -1;
  // air-path return to test for visibility: origin, direction and distance
  // to the sensor, its cell, fixed-point energy and outcome record slot
  bool has_air = false;
  float aox = 0, aoy = 0, aoz = 0, asx = 0, asy = 0, asz = 0, adist = 0;
  uint32_t acell = 0, aslot = 0xffffffffu;
  unsigned long long aqv = 0;
};

// Interaction of ray (a, b, c, m) with its closest hit (t bits, original
// triangle id, -1 for a miss): the record, the Snell/Fresnel split (float64
// energies), the standard-BRDF return over the beam window (Eq. 3-5), the
// range bin (Sec. III-B) and the two children with offset origins.  The
// bounce depth is that of the ray's heap id.  kAirPath: scans with the air-path
// flag also get the return along the air path (Sec. III-A, multi-path
// reflection) from hits at depth >= 1 in air, for a visibility ray to decide.
template <bool kAirPath>
__device__ __forceinline__ void shade_hit(const LevelArgs& A, const float4 a, const float4 b, const uint4 c,
                                          uint32_t m, uint32_t t_bits, int32_t hit, Shaded& o,
                                          const float4* normal = nullptr) {
  const uint32_t heap = m & 0xffu;
  const uint32_t medium = (m >> 8) & 0xffu;
  const uint32_t scan = m >> 16;
  const uint32_t depth = 31u - (uint32_t)__clz(heap);
  o.pid = c.z;
  o.hit = hit;
  const DevScan* S = A.scans + scan;
  // records per primary: the hit of every heap slot, then (air-path scans)
  // the air-path outcome of every slot
  const uint32_t nheap = (1u << S->max_b) - 1u;
  const size_t rbase = (size_t)o.pid * ((S->flags & kFlagAirPath) ? 2u * nheap : nheap);
  if (S->records) S->records[rbase + heap - 1] = hit >= 0 ? hit : -1;
  if (hit < 0) return;
  const float t = __uint_as_float(t_bits);
  const double E = __hiloint2double((int)c.y, (int)c.x);
  const float ox = a.x, oy = a.y, oz = a.z, L = a.w;
  const float dx = b.x, dy = b.y, dz = b.z;
  o.g = b.w;
  const float n_cur = medium == kAir ? 1.0f : A.mats[medium].n;
  const float4 ax = normal ? *normal : A.aux[hit];  // per original triangle
  const uint32_t mat = __float_as_uint(ax.w);
  const DevMaterial M = A.mats[mat];
  const float dn = dot3(dx, dy, dz, ax.x, ax.y, ax.z);
  const bool entering = dn < 0.0f;
  const float nfx = entering ? ax.x : -ax.x;
  const float nfy = entering ? ax.y : -ax.y;
  const float nfz = entering ? ax.z : -ax.z;
  const float dnf = dot3(dx, dy, dz, nfx, nfy, nfz);
  const float cosi = -dnf;
  const float k2 = 2.0f * dnf;
  // children exist below the last bounce level of the ray's scan; the
  // reflected direction is normalised only where a child or the air path
  // uses it (the last level skips both directions)
  const bool kids = depth + 1 < S->max_b;
  bool need_rd = kids;
  if constexpr (kAirPath) need_rd = need_rd || ((S->flags & kFlagAirPath) && depth >= 1u && medium == kAir);
  o.rdx = dx - k2 * nfx;
  o.rdy = dy - k2 * nfy;
  o.rdz = dz - k2 * nfz;
  if (need_rd) normalize3(o.rdx, o.rdy, o.rdz);
  double R, T;
  const double ci = (double)cosi;
  bool refract = false;
  uint32_t t_medium = kAir;
  if (M.kind == 0u || M.kind == 3u) {
    const float n1 = n_cur, n2 = entering ? M.n : 1.0f;
    const float eta = n1 / n2;
    const float kappa = 1.0f - (eta * eta) * (1.0f - cosi * cosi);
    if (kappa < 0.0f) {
      R = 1.0;
      T = 0.0;
    } else {
      if (kids) {
        const float cost = sqrtf(kappa);
        const float aa = eta * cosi - cost;
        const float ex = eta * dx, ey = eta * dy, ez = eta * dz;
        o.tdx = ex + aa * nfx;
        o.tdy = ey + aa * nfy;
        o.tdz = ez + aa * nfz;
        normalize3(o.tdx, o.tdy, o.tdz);
      }
      refract = true;
      t_medium = entering ? mat : kAir;
      if (M.kind == 3u) {
        // Cook-Torrance: a fixed reflected share, the rest refracts
        R = (double)M.refl;
      } else {
        const double N1 = n1, N2 = n2;
        const double e = N1 / N2;
        const double k64 = 1.0 - e * e * (1.0 - ci * ci);
        const double ct = sqrt(k64 > 0.0 ? k64 : 0.0);
        const double dsum = N1 * ci + N2 * ct, psum = N2 * ci + N1 * ct;
        if (dsum == 0.0 || psum == 0.0) {
          R = 1.0;
        } else {
          const double rs = (N1 * ci - N2 * ct) / dsum;
          const double rp = (N2 * ci - N1 * ct) / psum;
          R = 0.5 * (rs * rs + rp * rp);
        }
      }
      T = 1.0 - R;
    }
  } else {
    R = (double)M.refl;
    T = 0.0;
  }
  double w;
  if (S->flags & 8u) {
    w = 1.0;
  } else if (M.kind == 3u) {
    w = ct_return(M, nfx, nfy, nfz, dx, dy, dz, -dx, -dy, -dz);
  } else {
    double cw = 2.0 * ci * ci - 1.0;
    if (cw < 0.0) cw = 0.0;
    // cw - 1 = -2 (1 - cos)(1 + cos), accurate near the specular direction
    const float u = -2.0f * ((1.0f - cosi) * (1.0f + cosi));
    w = M.a + M.beta * cw + M.s * (double)lobe_pow(u, M.C);
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
  }
  const double e_ret = E * R * w;
  o.range = L + n_cur * t;
  const float q = o.range / S->bin_size;
  const uint32_t col = o.pid / S->n_s;
  if (q < (float)S->n_bins) {
    const uint32_t bin = (uint32_t)q;
    o.qv = __double2ull_rn(e_ret * (double)o.g * kFixedScale);
    if (o.qv) {
      o.cell = (uint32_t)(S->acc_base + (uint64_t)col * S->n_bins + bin);
      o.has_q = true;
    }
  }
  const float px = ox + t * dx, py = oy + t * dy, pz = oz + t * dz;
  double e_air = 0.0;
  if constexpr (kAirPath) {
    if ((S->flags & kFlagAirPath) && depth >= 1u && medium == kAir) {
      // from the reflected child's offset origin straight to the sensor
      const float aox = offset1(px, nfx), aoy = offset1(py, nfy), aoz = offset1(pz, nfz);
      const float vx = S->pos[0] - aox, vy = S->pos[1] - aoy, vz = S->pos[2] - aoz;
      const float dist = sqrtf(dot3(vx, vy, vz, vx, vy, vz));
      float sx = 0.0f, sy = 0.0f, sz = 0.0f;
      if (dist > 0.0f) {
        sx = vx / dist;
        sy = vy / dist;
        sz = vz / dist;
      }
      if (dist > 0.0f && dot3(sx, sy, sz, nfx, nfy, nfz) > 0.0f) {
        double w_air;
        if (S->flags & 8u) {
          w_air = 1.0;
        } else if (M.kind == 3u) {
          w_air = ct_return(M, nfx, nfy, nfz, dx, dy, dz, sx, sy, sz);
        } else {
          double ca = (double)o.rdx * sx + (double)o.rdy * sy + (double)o.rdz * sz;
          ca = ca < 0.0 ? 0.0 : (ca > 1.0 ? 1.0 : ca);
          w_air = M.a + M.beta * ca + M.s * (double)lobe_pow((float)(ca - 1.0), M.C);
          w_air = w_air < 0.0 ? 0.0 : (w_air > 1.0 ? 1.0 : w_air);
        }
        e_air = E * R * w_air;
        const double room = E * R - e_ret;
        if (e_air > room) e_air = room;
        double g_air = 1.0;
        if (S->flags & 1u) {
          // angle between the column's beam axis and the arrival direction
          const double phi = 2.0 * M_PI * (double)col / (double)S->n_az;
          const double c0 = cos(phi), s0 = sin(phi);
          const double ax0 = S->R[0] * c0 + S->R[1] * s0;
          const double ax1 = S->R[3] * c0 + S->R[4] * s0;
          const double ax2 = S->R[6] * c0 + S->R[7] * s0;
          const double w0 = (double)aox - (double)S->pos[0];
          const double w1 = (double)aoy - (double)S->pos[1];
          const double w2 = (double)aoz - (double)S->pos[2];
          const double x0 = ax1 * w2 - ax2 * w1, x1 = ax2 * w0 - ax0 * w2, x2 = ax0 * w1 - ax1 * w0;
          const double alpha = atan2(sqrt(x0 * x0 + x1 * x1 + x2 * x2), ax0 * w0 + ax1 * w1 + ax2 * w2);
          if (S->sigma_r > 0.0) {
            const double z = alpha / S->sigma_r;
            g_air = exp(-0.5 * z * z);
          } else {
            g_air = alpha == 0.0 ? 1.0 : 0.0;
          }
        }
        const float range_air = (o.range + dist) * 0.5f;
        const float qa = range_air / S->bin_size;
        const size_t aslot = rbase + nheap + heap - 1;
        if (qa < (float)S->n_bins) {
          o.aqv = __double2ull_rn(e_air * g_air * kFixedScale);
          // a visibility ray only where it can add energy or a record is kept
          if (o.aqv || S->records) {
            o.has_air = true;
            o.aox = aox;
            o.aoy = aoy;
            o.aoz = aoz;
            o.asx = sx;
            o.asy = sy;
            o.asz = sz;
            o.adist = dist;
            o.acell = (uint32_t)(S->acc_base + (uint64_t)col * S->n_bins + (uint32_t)qa);
            o.aslot = S->records ? (uint32_t)aslot : 0xffffffffu;
          }
        } else if (S->records) {
          S->records[aslot] = 2;
        }
      }
    }
  }
  if (kids) {
    const double ecut = (double)S->e_cut;
    o.e_refl = E * R - e_ret - e_air;
    o.e_refr = refract ? E * T : 0.0;
    if (o.e_refl > ecut) {
      o.has_r = true;
      o.rox = offset1(px, nfx);
      o.roy = offset1(py, nfy);
      o.roz = offset1(pz, nfz);
    }
    if (refract && o.e_refr > ecut) {
      o.has_t = true;
      o.tox = offset1(px, -nfx);
      o.toy = offset1(py, -nfy);
      o.toz = offset1(pz, -nfz);
    }
  }
  o.r_meta = (scan << 16) | (medium << 8) | (2u * heap);
  o.t_meta = (scan << 16) | (t_medium << 8) | (2u * heap + 1u);
}

// Interaction at the hit of every ray of the level (Sec. III-A): Snell and
// Fresnel split, the retrace return through the beam window of the standard
// BRDF, range binning (Sec. III-B) and the two children.
// Register budgets for occupancy: the kernel mostly waits on its loads, and
// more resident waves hide more of that wait.  The closest-hit form keeps to
// 80 registers, six waves per SIMD (three 512-lane blocks per CU instead of
// two); the air-path form to 168, three waves per SIMD (three 256-lane blocks
// instead of two).  The closest-hit form spills one register to scratch.
template <bool kCount, bool kAirPath>
__global__ void __launch_bounds__(shade_block(kAirPath)) __attribute__((amdgpu_waves_per_eu(kAirPath ? 3 : 6)))
k_shade(LevelArgs A) {
  constexpr int kShadeLanes = shade_block(kAirPath);
  // returns of the block's rays are summed in an LDS hash table keyed by
  // accumulator cell and flushed with one global atomic per cell at the end;
  // the block works on a contiguous range of the level, whose rays mostly
  // share azimuths and so few cells
  __shared__ uint32_t h_key[kHashSlots];
  __shared__ unsigned long long h_val[kHashSlots];
  // per-wave child counts and the block's queue bases, double-buffered by
  // block step so that one step's readers never race the next step's writers
  __shared__ uint32_t s_cnt[2][kShadeLanes / 64][3];
  __shared__ uint32_t s_base[2], s_abase[2];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t n_in = min(A.counters[kCtrCount + A.depth], A.cap);
  for (uint32_t i = threadIdx.x; i < kHashSlots; i += kShadeLanes) {
    h_key[i] = kHashEmpty;
    h_val[i] = 0ull;
  }
  __syncthreads();
  const uint32_t per_block = ((n_in + gridDim.x - 1) / gridDim.x + kShadeLanes - 1) / kShadeLanes * kShadeLanes;
  const uint32_t begin = min(blockIdx.x * per_block, n_in);
  const uint32_t end = min(begin + per_block, n_in);
  uint32_t cnt_hits = 0;
  uint32_t par = 0;
  // the ray, its hit and the hit triangle's normal are loaded at the top of
  // the step: the other resident waves cover their latency (loading one
  // step ahead held 19 more registers and cost spills at this occupancy)
  for (uint32_t base = begin; base < end; base += kShadeLanes, par ^= 1u) {
    const uint32_t idx = base + threadIdx.x;
    const bool active = idx < end;
    uint2 h = make_uint2(0u, 0xffffffffu);
    float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a, nrm = a;
    uint4 c = make_uint4(0u, 0u, 0u, 0u);
    uint32_t m = 0;
    if (active) {
      h = A.hits[idx];
      a = A.in.a[idx];
      b = A.in.b[idx];
      c = A.in.c[idx];
      m = A.in.m[idx];
      if ((int32_t)h.y >= 0) nrm = A.aux[h.y];
    }
    Shaded o;
    if (active) {
      const int32_t hit = (int32_t)h.y;
      shade_hit<kAirPath>(A, a, b, c, m, h.x, hit, o, &nrm);
      if (kCount && hit >= 0) ++cnt_hits;
    }
    const bool has_q = o.has_q, has_r = o.has_r, has_t = o.has_t;
    const uint32_t cell = o.cell;
    const unsigned long long qv = o.qv;
    // ---- return into the block's table (global atomic if its probe fails)
    if (has_q) {
      uint32_t h = (cell * 2654435761u) >> (32 - kHashBits);
      bool done = false;
#pragma unroll 1
      for (int probe = 0; probe < 8 && !done; ++probe) {
        const uint32_t prev = atomicCAS(&h_key[h], kHashEmpty, cell);
        if (prev == kHashEmpty || prev == cell) {
          atomicAdd(&h_val[h], qv);
          done = true;
        }
        h = (h + 1u) & (kHashSlots - 1u);
      }
      if (!done) atomicAdd(A.acc + cell, qv);
    }

    // ---- children (and visibility rays): one atomic per block iteration for
    // every kind; the last level of a launch without the air path has none
    if (kAirPath || A.depth + 1 < A.levels) {
      const uint64_t mr = __ballot(has_r);
      const uint64_t mt = __ballot(has_t);
      const uint64_t ma = kAirPath ? __ballot(o.has_air) : 0ull;
      const uint32_t nr = (uint32_t)__popcll(mr);
      const uint32_t nt = (uint32_t)__popcll(mt);
      if (lane == 0) {
        s_cnt[par][wid][0] = nr;
        s_cnt[par][wid][1] = nt;
        s_cnt[par][wid][2] = (uint32_t)__popcll(ma);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t total = 0, total_a = 0;
        for (uint32_t w = 0; w < kShadeLanes / 64; ++w) {
          total += s_cnt[par][w][0] + s_cnt[par][w][1];
          total_a += s_cnt[par][w][2];
        }
        s_base[par] = total ? atomicAdd(A.counters + kCtrCount + A.depth + 1, total) : 0u;
        if (kAirPath) s_abase[par] = total_a ? atomicAdd(A.counters + kCtrShadow, total_a) : 0u;
      }
      __syncthreads();
      // buffer `par` is written again two steps on, after every wave has passed
      // the next step's first barrier, so no third barrier is needed here
      uint32_t ob = s_base[par], oa = kAirPath ? s_abase[par] : 0u;
      for (uint32_t w = 0; w < wid; ++w) {
        ob += s_cnt[par][w][0] + s_cnt[par][w][1];
        if (kAirPath) oa += s_cnt[par][w][2];
      }
      if (kAirPath && o.has_air) {
        const uint32_t slot = oa + lane_prefix(ma);
        if (slot < A.shq_cap) {
          A.shq.a[slot] = make_float4(o.aox, o.aoy, o.aoz, o.adist);
          A.shq.b[slot] = make_float4(o.asx, o.asy, o.asz, __uint_as_float(o.aslot));
          A.shq.c[slot] = make_uint4((uint32_t)o.aqv, (uint32_t)(o.aqv >> 32), o.acell, (uint32_t)o.hit);
        } else {
          atomicOr(A.counters + kCtrOverflow, 1u);
        }
      }
      if (has_r) {
        const uint32_t slot = ob + lane_prefix(mr);
        if (slot < A.cap)
          put_ray(A.out, slot, o.rox, o.roy, o.roz, o.range, o.rdx, o.rdy, o.rdz, o.g, o.e_refl, o.pid,
                  (uint32_t)o.hit, o.r_meta);
        else
          atomicOr(A.counters + kCtrOverflow, 1u);
      }
      if (has_t) {
        const uint32_t slot = ob + nr + lane_prefix(mt);
        if (slot < A.cap)
          put_ray(A.out, slot, o.tox, o.toy, o.toz, o.range, o.tdx, o.tdy, o.tdz, o.g, o.e_refr, o.pid,
                  (uint32_t)o.hit, o.t_meta);
        else
          atomicOr(A.counters + kCtrOverflow, 1u);
      }
    }
  }
  // ---- flush the table
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHashSlots; i += kShadeLanes)
    if (h_key[i] != kHashEmpty) atomicAdd(A.acc + h_key[i], h_val[i]);
  if (kCount) atomicAdd(A.prof + 3, (unsigned long long)cnt_hits);
}

// ---------------------------------------------------------------- fused scan
// All bounce levels in one persistent launch.  Each wave runs its own
// wavefront loop over three kinds of step, chosen for the whole wave:
//   node step      every tracing lane visits one inner node (as k_trace);
//   triangle phase up to 64 queued leaves, one per lane (as k_trace);
//   shade phase    up to 64 finished rays from the wave's hit ring, one per
//                  lane: the interaction, the return added into the image
//                  accumulator with a 64-bit atomic, the children pushed on
//                  the wave's child pool.
// Idle lanes take children from the pool (last in, first out) and only when
// it is empty new primaries from the level-0 queue, so lanes stay busy across
// levels and the only tail is the end of the scan.  The hit ring and child
// pool are private to the wave (workspace memory, written and read by the
// same wave, ordered with workgroup-scope fences), so waves never wait on
// each other.  Every ray is traced and shaded exactly as in the
// level-by-level kernels, so the images are identical.
template <bool kCount>
__global__ void __launch_bounds__(kTraceBlock) k_scan(LevelArgs A) {
  __shared__ int32_t lds_stack[kStack * kTraceBlock];
  __shared__ uint32_t lds_leaf[kTraceBlock / 64][kLeafRing];
  __shared__ uint8_t lds_own[kTraceBlock / 64][kLeafRing];
  __shared__ unsigned long long lds_best[kTraceBlock];
  int32_t* stk = lds_stack + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wib = threadIdx.x >> 6;
  const uint32_t wave_base = threadIdx.x - lane;
  const uint32_t n_in = min(A.counters[kCtrCount], A.cap);
  uint32_t seg = blockIdx.x & (kCtrSegs - 1u), seg_tries = 0;  // claim_rays state (level 0's cursors)
  uint32_t* const seg_cur = A.counters + kCtrCursor;
  const Node4* __restrict__ nodes = A.nodes;
  const float4* __restrict__ tris = A.tris;
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t spill_stride = gridDim.x * blockDim.x;
  const uint32_t tri_batch = min(max(A.tri_batch, 1u), 64u);
  const uint32_t shade_batch = min(max(A.shade_batch, 1u), 64u);
  const uint32_t wave_id = blockIdx.x * (kTraceBlock / 64) + wib;
  // wave-private child pool (wq_pool entries) and hit ring (wq_hits, a power
  // of two), four float4 per entry: (o, L), (d, g), (E lo, E hi, pid, excl),
  // (meta, t bits, hit, 0)
  float4* const pool = A.wq + (size_t)wave_id * (A.wq_pool + A.wq_hits) * 4u;
  float4* const hring = pool + (size_t)A.wq_pool * 4u;

  bool valid = false, exhausted = false;
  uint32_t pool_next = 0, pool_end = 0;     // wave-uniform: claimed primaries
  uint32_t ring_head = 0, ring_tail = 0;    // wave-uniform: leaf ring
  uint32_t hit_head = 0, hit_tail = 0;      // wave-uniform: hit ring
  uint32_t pool_n = 0;                      // wave-uniform: children in the pool
  uint32_t n_depth[kMaxLevels] = {};    // wave-uniform: children created per depth
  uint32_t visits = 0, excl = 0xffffffffu, last_pos = 0;
  float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, best_t = 0, ray_L = 0, ray_g = 0;
  uint4 ray_c = make_uint4(0u, 0u, 0u, 0u);
  uint32_t ray_m = 0;
  RayBox rb{};
  int32_t cur = 0;
  int sp = 0;
  bool trav_done = false;
  uint32_t cnt_nodes = 0, cnt_tris = 0, cnt_rays = 0, cnt_hits = 0, cnt_pool_max = 0;

  auto start_ray = [&](const float4 a, const float4 b, const uint4 c, uint32_t m) {
    excl = c.w;
    const uint32_t medium = (m >> 8) & 0xffu;
    const float n_cur = medium == kAir ? 1.0f : A.mats[medium].n;
    best_t = (A.scans[m >> 16].r_max - a.w) / n_cur;
    lds_best[threadIdx.x] = ((unsigned long long)__float_as_uint(best_t) << 32) | 0xffffffffull;
    ox = a.x;
    oy = a.y;
    oz = a.z;
    dx = b.x;
    dy = b.y;
    dz = b.z;
    ray_L = a.w;
    ray_g = b.w;
    ray_c = c;
    ray_m = m;
    ray_box_setup(ox, oy, oz, dx, dy, dz, rb);
    cur = 0;
    sp = 0;
    visits = 0;
    last_pos = ring_head;
    trav_done = false;
    valid = true;
    if (kCount) ++cnt_rays;
  };

  for (;;) {
    // ---- refill idle lanes: children of this wave first, then primaries
    uint64_t idle = __ballot(!valid);
    if (pool_n > 0 && idle) {
      const uint32_t take = min((uint32_t)__popcll(idle), pool_n);
      const uint32_t rank = lane_prefix(idle);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      if (!valid && rank < take) {
        const float4* e = pool + (size_t)(pool_n - 1u - rank) * 4u;
        const float4 a = e[0], b = e[1];
        const uint4 c = reinterpret_cast<const uint4*>(e)[2];
        const uint32_t m = reinterpret_cast<const uint4*>(e)[3].x;
        start_ray(a, b, c, m);
      }
      pool_n -= take;
      idle = __ballot(!valid);
    }
    if (!exhausted && pool_n == 0 && (uint32_t)__popcll(idle) >= A.refill) {
#pragma unroll 1
      for (int pass = 0; pass < 2 && idle; ++pass) {
        if (pool_next >= pool_end &&
            !claim_rays(seg_cur, n_in, A.pool, lane, seg, seg_tries, pool_next, pool_end)) {
          exhausted = true;
          break;
        }
        const uint32_t take = min((uint32_t)__popcll(idle), pool_end - pool_next);
        const uint32_t rank = lane_prefix(idle);
        if (!valid && rank < take) {
          const uint32_t my = pool_next + rank;
          start_ray(A.in.a[my], A.in.b[my], A.in.c[my], A.in.m[my]);
        }
        pool_next += take;
        idle = __ballot(!valid);
      }
    }
    const uint64_t live = __ballot(valid);
    const uint32_t hits_q = hit_head - hit_tail;
    if (live == 0ull && hits_q == 0u && pool_n == 0u && exhausted) break;

    const uint64_t walking = __ballot(valid && !trav_done);
    const uint32_t queued = ring_head - ring_tail;
    const bool shade_phase = hits_q >= shade_batch || hits_q + 64u > A.wq_hits ||
                             (hits_q > 0u && live == 0ull);
    const bool tri_phase = !shade_phase &&
                           (queued >= tri_batch ||
                            (queued > 0 && (walking == 0ull || queued + 4u * (uint32_t)__popcll(walking) > kLeafRing)));
    if (shade_phase) {
      // ---- interactions of up to 64 finished rays, one per lane
      const uint32_t n = min(hits_q, 64u);
      const bool take = lane < n;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      Shaded o;
      uint32_t child_depth = 0;
      if (take) {
        const float4* e = hring + (size_t)((hit_tail + lane) & (A.wq_hits - 1u)) * 4u;
        const float4 a = e[0], b = e[1];
        const uint4 c = reinterpret_cast<const uint4*>(e)[2];
        const uint4 d = reinterpret_cast<const uint4*>(e)[3];
        shade_hit<false>(A, a, b, c, d.x, d.y, (int32_t)d.z, o);
        if (o.has_q) atomicAdd(A.acc + o.cell, o.qv);
        child_depth = 32u - (uint32_t)__clz(d.x & 0xffu);  // depth of the ray + 1
        if (kCount && o.hit >= 0) ++cnt_hits;
      }
      hit_tail += n;
      const uint64_t mr = __ballot(take && o.has_r);
      const uint64_t mt = __ballot(take && o.has_t);
      const uint32_t nr = (uint32_t)__popcll(mr), nt = (uint32_t)__popcll(mt);
      if (pool_n + nr + nt <= A.wq_pool) {
        if (take && o.has_r) {
          float4* e = pool + (size_t)(pool_n + lane_prefix(mr)) * 4u;
          e[0] = make_float4(o.rox, o.roy, o.roz, o.range);
          e[1] = make_float4(o.rdx, o.rdy, o.rdz, o.g);
          reinterpret_cast<uint4*>(e)[2] = make_uint4((uint32_t)__double2loint(o.e_refl),
                                                      (uint32_t)__double2hiint(o.e_refl), o.pid, (uint32_t)o.hit);
          reinterpret_cast<uint4*>(e)[3] = make_uint4(o.r_meta, 0u, 0u, 0u);
        }
        if (take && o.has_t) {
          float4* e = pool + (size_t)(pool_n + nr + lane_prefix(mt)) * 4u;
          e[0] = make_float4(o.tox, o.toy, o.toz, o.range);
          e[1] = make_float4(o.tdx, o.tdy, o.tdz, o.g);
          reinterpret_cast<uint4*>(e)[2] = make_uint4((uint32_t)__double2loint(o.e_refr),
                                                      (uint32_t)__double2hiint(o.e_refr), o.pid, (uint32_t)o.hit);
          reinterpret_cast<uint4*>(e)[3] = make_uint4(o.t_meta, 0u, 0u, 0u);
        }
        pool_n += nr + nt;
#pragma unroll
        for (uint32_t d = 1; d < kMaxLevels; ++d)
          n_depth[d] += (uint32_t)__popcll((mr | mt) & __ballot(take && child_depth == d)) +
                        (uint32_t)__popcll(mr & mt & __ballot(take && child_depth == d));
        if (kCount) cnt_pool_max = max(cnt_pool_max, pool_n);
      } else if (nr + nt > 0u && lane == 0) {
        atomicOr(A.counters + kCtrOverflow, 1u);  // pool full: children dropped, scan reports it
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    } else if (tri_phase) {
      const uint32_t n = min(queued, 64u);
      const bool take = lane < n;
      const uint32_t pos = (ring_tail + lane) & (kLeafRing - 1u);
      const uint32_t ref = take ? lds_leaf[wib][pos] : 0u;
      const int own = take ? (int)lds_own[wib][pos] : (int)lane;
      const float rox = __shfl(ox, own), roy = __shfl(oy, own), roz = __shfl(oz, own);
      const float rdx = __shfl(dx, own), rdy = __shfl(dy, own), rdz = __shfl(dz, own);
      const uint32_t rexcl = __shfl(excl, own);
      if (take) {
        unsigned long long cb = lds_best[wave_base + own];
        float tmax = __uint_as_float((uint32_t)(cb >> 32));
        const uint32_t start = leaf_start((int32_t)ref), count = leaf_count((int32_t)ref);
#pragma unroll 1
        for (uint32_t k = 0; k < count; ++k) {
          const uint32_t li = start + k;
          const float4 ta = tris[3 * li + 0];
          const uint32_t orig = __float_as_uint(ta.w);
          if (orig == rexcl) continue;
          if (kCount) ++cnt_tris;
          const float4 e1 = tris[3 * li + 1];
          const float4 e2 = tris[3 * li + 2];
          float t;
          if (ray_tri(rox, roy, roz, rdx, rdy, rdz, ta.x, ta.y, ta.z, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z,
                      tmax, t)) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | orig;
            if (key < cb) {
              atomicMin(&lds_best[wave_base + own], key);
              cb = key;
              tmax = t;
            }
          }
        }
      }
      ring_tail += n;
      __builtin_amdgcn_wave_barrier();
      if (valid) best_t = __uint_as_float((uint32_t)(lds_best[threadIdx.x] >> 32));
    } else {
      uint32_t leaves = 0;
      int32_t lref[4] = {0, 0, 0, 0};
      if (valid && !trav_done) {
        const int32_t top = stk[min(max(sp - 1, 0), kStack - 1) * kTraceBlock];
        if (cur == kEmpty) {
          if (sp > 0) {
            --sp;
            cur = sp < kStack ? top : A.spill[(size_t)(sp - kStack) * spill_stride + gtid];
          } else {
            trav_done = true;
          }
        }
        if (!trav_done) {
          const float4* np = reinterpret_cast<const float4*>(nodes + cur);
          const float4 w0 = np[0];
          const uint4 w1 = reinterpret_cast<const uint4*>(np)[1];
          const uint4 w2 = reinterpret_cast<const uint4*>(np)[2];
          const int4 w3 = reinterpret_cast<const int4*>(np)[3];
          if (kCount) ++cnt_nodes;
          float tn[4];
          const uint32_t mask = node4_boxes(w0, w1, w2, w3, rb, best_t, tn);
          const int32_t ref[4] = {w3.x, w3.y, w3.z, w3.w};
          float key[4];
          int32_t val[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool h = (mask >> j) & 1u;
            const bool inner = h && ref[j] >= 0;
            if (h && ref[j] < 0) leaves |= 1u << j;
            lref[j] = ref[j];
            key[j] = inner ? tn[j] : -INFINITY;
            val[j] = inner ? ref[j] : kEmpty;
          }
#define RR_CX(i, j)                     \
  if (key[j] > key[i]) {                \
    const float tk = key[i];            \
    key[i] = key[j];                    \
    key[j] = tk;                        \
    const int32_t tv = val[i];          \
    val[i] = val[j];                    \
    val[j] = tv;                        \
  }
          RR_CX(0, 1) RR_CX(2, 3) RR_CX(0, 2) RR_CX(1, 3) RR_CX(1, 2)
#undef RR_CX
          const int h = __popc(mask & ~leaves);
          if (sp + 3 <= kStack) {
            stk[(sp + 0) * kTraceBlock] = val[0];
            stk[(sp + 1) * kTraceBlock] = val[1];
            stk[(sp + 2) * kTraceBlock] = val[2];
            sp += h > 1 ? h - 1 : 0;
          } else {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              if (j < h - 1 && sp < kStack + kSpill) {
                if (sp < kStack)
                  stk[sp * kTraceBlock] = val[j];
                else
                  A.spill[(size_t)(sp - kStack) * spill_stride + gtid] = val[j];
                ++sp;
              }
            }
          }
          cur = h == 0 ? kEmpty : h == 1 ? val[0] : h == 2 ? val[1] : h == 3 ? val[2] : val[3];
          if (++visits > A.n_nodes) trav_done = true;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool want = (leaves >> j) & 1u;
        const uint64_t m = __ballot(want);
        if (want) {
          const uint32_t p = ring_head + lane_prefix(m);
          lds_leaf[wib][p & (kLeafRing - 1u)] = (uint32_t)lref[j];
          lds_own[wib][p & (kLeafRing - 1u)] = (uint8_t)lane;
          last_pos = p + 1u;
        }
        ring_head += (uint32_t)__popcll(m);
      }
    }
    __builtin_amdgcn_wave_barrier();

    // ---- finished rays into the hit ring (room for 64 is kept free)
    const bool fin = valid && trav_done && (int32_t)(ring_tail - last_pos) >= 0;
    const uint64_t fm = __ballot(fin);
    if (fin) {
      const unsigned long long bst = lds_best[threadIdx.x];
      float4* e = hring + (size_t)((hit_head + lane_prefix(fm)) & (A.wq_hits - 1u)) * 4u;
      e[0] = make_float4(ox, oy, oz, ray_L);
      e[1] = make_float4(dx, dy, dz, ray_g);
      reinterpret_cast<uint4*>(e)[2] = ray_c;
      reinterpret_cast<uint4*>(e)[3] = make_uint4(ray_m, (uint32_t)(bst >> 32), (uint32_t)bst, 0u);
      valid = false;
    }
    hit_head += (uint32_t)__popcll(fm);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  }
  if (lane == 0) {
#pragma unroll
    for (uint32_t d = 1; d < kMaxLevels; ++d)
      if (n_depth[d]) atomicAdd(A.counters + kCtrCount + d, n_depth[d]);
  }
  if (kCount) {
    atomicAdd(A.prof + 0, (unsigned long long)cnt_nodes);
    atomicAdd(A.prof + 1, (unsigned long long)cnt_tris);
    atomicAdd(A.prof + 2, (unsigned long long)cnt_rays);
    atomicAdd(A.prof + 3, (unsigned long long)cnt_hits);
    if (lane == 0) atomicMax(A.prof + kProfPoolMax, (unsigned long long)cnt_pool_max);
  }
}

// ---------------------------------------------------------------- helpers
struct Blob {
  uint32_t n_words;
  uint32_t w[760];
};

__global__ void k_put(uint32_t* dst, Blob b) {
  for (uint32_t i = threadIdx.x; i < b.n_words; i += blockDim.x) dst[i] = b.w[i];
}

__global__ void k_clear(unsigned long long* acc, size_t n_acc, uint32_t* counters, uint32_t count0) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = i; j < n_acc; j += stride) acc[j] = 0ull;
  if (i < (size_t)kCtrWords) counters[i] = (i == (size_t)kCtrCount) ? count0 : 0u;
}

// Random 64-byte gathers over a working set (a bandwidth probe with the
// access pattern of node and triangle fetches): each group of four lanes
// reads one 64-byte row per step at a hashed index, coalesced as 4 x 16 B.
__global__ void k_gather(const float4* buf, uint32_t n_rows, uint32_t steps, float* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t group = t >> 2, part = t & 3u;
  float acc = 0.0f;
  uint32_t h = group * 2654435761u + 0x9E3779B9u;
#pragma unroll 4
  for (uint32_t i = 0; i < steps; ++i) {
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    const float4 v = buf[(size_t)(h % n_rows) * 4u + part];
    acc += v.x + v.y + v.z + v.w;
  }
  out[t] = acc;
}

hipError_t launch_gather(const float4* buf, uint32_t n_rows, uint32_t steps, float* out, uint32_t threads,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(threads / 256u), dim3(256), 0, st, buf, n_rows, steps, out);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) p[j] = v;
}

__global__ void k_finalize(const DevScan* scans, const unsigned long long* acc) {
  const DevScan& s = scans[blockIdx.y];
  size_t n = (size_t)s.n_az * s.n_bins;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
    s.image[j] = (float)((double)acc[s.acc_base + j] * kFixedInv);
}

hipError_t put_blob(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const uint32_t* w = static_cast<const uint32_t*>(src);
  size_t words = bytes / 4;
  uint32_t* d = static_cast<uint32_t*>(dst);
  Blob b;
  for (size_t off = 0; off < words; off += 760) {
    size_t n = words - off < 760 ? words - off : 760;
    b.n_words = (uint32_t)n;
    for (size_t i = 0; i < n; ++i) b.w[i] = w[off + i];
    hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, d + off, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_clear(unsigned long long* acc, size_t n_acc, uint32_t* counters, uint32_t count0,
                        hipStream_t st) {
  size_t blocks = (n_acc + 255) / 256;
  if (blocks < (size_t)(kCtrWords + 255) / 256) blocks = (size_t)(kCtrWords + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)blocks), dim3(256), 0, st, acc, n_acc, counters, count0);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_raygen(const LevelArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_raygen, dim3(grid ? grid : 1), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_trace(const LevelArgs& a, uint32_t grid, bool help, hipStream_t st) {
  const dim3 g(grid ? grid : 1), b(kTraceBlock);
  if (a.nodes8) {
    if (a.prof)
      hipLaunchKernelGGL(k_trace8<true>, g, b, 0, st, a);
    else
      hipLaunchKernelGGL(k_trace8<false>, g, b, 0, st, a);
    return hipGetLastError();
  }
  if (a.prof && help)
    hipLaunchKernelGGL((k_trace<true, false, true>), g, b, 0, st, a);
  else if (a.prof)
    hipLaunchKernelGGL((k_trace<true, false, false>), g, b, 0, st, a);
  else if (help)
    hipLaunchKernelGGL((k_trace<false, false, true>), g, b, 0, st, a);
  else
    hipLaunchKernelGGL((k_trace<false, false, false>), g, b, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_shadow(const LevelArgs& a, uint32_t grid, bool help, hipStream_t st) {
  if (help)
    hipLaunchKernelGGL((k_trace<false, true, true>), dim3(grid ? grid : 1), dim3(kTraceBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_trace<false, true, false>), dim3(grid ? grid : 1), dim3(kTraceBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scan(const LevelArgs& a, uint32_t grid, hipStream_t st) {
  const dim3 g(grid ? grid : 1), b(kTraceBlock);
  if (a.prof)
    hipLaunchKernelGGL(k_scan<true>, g, b, 0, st, a);
  else
    hipLaunchKernelGGL(k_scan<false>, g, b, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_shade(const LevelArgs& a, uint32_t grid, hipStream_t st) {
  const dim3 g(grid ? grid : 1), b(shade_block(a.air));
  if (a.air) {
    if (a.prof)
      hipLaunchKernelGGL((k_shade<true, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_shade<false, true>), g, b, 0, st, a);
  } else {
    if (a.prof)
      hipLaunchKernelGGL((k_shade<true, false>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_shade<false, false>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const DevScan* scans, uint32_t n_scans, const unsigned long long* acc,
                           uint32_t max_cells, hipStream_t st) {
  uint32_t blocks = (max_cells + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_finalize, dim3(blocks, n_scans), dim3(256), 0, st, scans, acc);
  return hipGetLastError();
}

}  // namespace rr
