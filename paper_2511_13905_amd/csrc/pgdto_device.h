// Device-side building blocks shared by the projection kernels: loads,
// float64 helpers, cross-workgroup publication, workgroup and grid
// reductions, the grid barrier, tile geometry, the 1-D bracket search control
// (Algorithm 1), the automatic penalty and stated-error rules, and the step
// rule of Algorithm 3.
#pragma once

#include "pgdto_internal.h"
#include "pgdto_ctx.h"

#include <math.h>

#include <type_traits>

namespace pgdto {


enum Phase : int32_t {
  PH_PGD_R = 1,   // Alg. 3 reductions (step size, direction, a.rho_t)
  PH_ZERO = 2,    // lam = 0: h(0), slope, bracket end (pgd: also writes d_t, rho~)
  PH_SEARCH = 3,  // 1-D bracket search pass (Alg. 1)
  PH_STAGE1 = 4,  // coupled: lockstep single-row searches (Alg. 2 Stage 1)
  PH_CHECK = 5,   // coupled: candidate feasibility (+ Newton evaluation at lam0)
  PH_NEWTON = 6,  // coupled: h and J at a trial multiplier
  PH_FINAL = 7,   // write x, residuals, free count, stop-test norms
  PH_DONE = 8
};

enum SegState : int32_t { SEG_SEARCH = 0, SEG_DONE = 1 };

// ------------------------------------------------------------------ loads

template <typename T> struct VT;
template <> struct VT<float> { static constexpr int N = 4; };
template <> struct VT<double> { static constexpr int N = 2; };

// Global-address-space views of generic pointers (the pointers come from the
// LDS copy of the descriptor; without the cast the compiler emits flat
// accesses, which also wait on the LDS counter).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr_w(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// NT: a non-temporal load.  A pass of the Algorithm 3 step batch reads each
// whole line once, so its loads need not displace other lines in the
// caches: for that byte mix a plain kernel reaches 6.6 TB/s with them against
// 6.0 TB/s with ordinary loads.  Where one load instruction covers only part
// of each line (the wide kernel's 64-byte row segments), ordinary loads keep
// the line for the instruction that reads its other half.
template <typename T, bool NT = false>
__device__ __forceinline__ void ld_vec_whole(const __attribute__((address_space(1))) T* p, int64_t e0, T* o) {
  if constexpr (sizeof(T) == 4) {
    const auto* q0 = reinterpret_cast<const __attribute__((address_space(1))) f32x4*>(p + e0);
    f32x4 q;
    if constexpr (NT) q = __builtin_nontemporal_load(q0); else q = *q0;
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
  } else {
    const auto* q0 = reinterpret_cast<const __attribute__((address_space(1))) f64x2*>(p + e0);
    f64x2 q;
    if constexpr (NT) q = __builtin_nontemporal_load(q0); else q = *q0;
    o[0] = q.x; o[1] = q.y;
  }
}

// One vector slot near the array's end: V element loads from e0, each
// address clamped into [0, n) (n >= 1 on every launch) and elements at or
// past n replaced by 0.  Every lane issues exactly V loads with no branch, so
// the compiler can count the loads in flight and wait only for older ones.
template <typename T>
__device__ __forceinline__ void ld_vec_tail(const __attribute__((address_space(1))) T* p, int64_t e0, int64_t n, T* o) {
  constexpr int V = VT<T>::N;
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const T v = p[min(e0 + k, n - 1)];
    o[k] = (e0 + k < n) ? v : (T)0;
  }
}

// One vector slot, the whole-vector or the tail form chosen per lane.
template <typename T, bool NT = false>
__device__ __forceinline__ void ld_vec(const T* __restrict__ p0, int64_t e0, int64_t n, bool, T* o) {
  const auto p = gptr(p0);
  if (e0 + VT<T>::N <= n) ld_vec_whole<T, NT>(p, e0, o);
  else ld_vec_tail<T>(p, e0, n, o);
}

// K vector slots of NS streams at once.  When every lane of the wave has all
// its K vectors inside the array (everywhere but near the array's end), one
// wave-uniform branch issues the K x NS 16-byte loads back to back with no
// other control flow, so they are all in flight together; a per-lane choice
// between a vector load and element loads into the same registers would make
// the compiler wait for each load before issuing the next.
template <typename T, int K, int NS, bool NT = false>
__device__ __forceinline__ void ld_slots(const T* const* ptrs, const int64_t* e0, int64_t n,
                                         T (&buf)[K][NS][VT<T>::N]) {
  constexpr int V = VT<T>::N;
  bool whole = true;
#pragma unroll
  for (int k = 0; k < K; ++k) whole = whole && (e0[k] + V <= n);
  if (__all(whole)) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < NS; ++q) ld_vec_whole<T, NT>(gptr(ptrs[q]), e0[k], buf[k][q]);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < NS; ++q) ld_vec_tail<T>(gptr(ptrs[q]), e0[k], n, buf[k][q]);
  }
}

// Streamed outputs (x, d_t, a materialized rho~) are written with
// non-temporal stores: they do not pile up as dirty lines in L2, which the
// release at the end of every pass (an L2 write-back) would otherwise flush.
template <typename T>
__device__ __forceinline__ void st_vec(T* __restrict__ p0, int64_t e0, uint32_t mask, bool full, const T* v) {
  const auto p = gptr_w(p0);
  if (full) {
    if constexpr (sizeof(T) == 4) {
      const f32x4 q = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(q, reinterpret_cast<__attribute__((address_space(1))) f32x4*>(p + e0));
    } else {
      const f64x2 q = {v[0], v[1]};
      __builtin_nontemporal_store(q, reinterpret_cast<__attribute__((address_space(1))) f64x2*>(p + e0));
    }
  } else {
#pragma unroll
    for (int k = 0; k < VT<T>::N; ++k)
      if (mask & (1u << k)) p[e0 + k] = v[k];
  }
}

template <typename T>
__device__ __forceinline__ double f64(T v) { return (double)v; }

__device__ __forceinline__ double clampd(double z, double lo, double hi) { return fmin(fmax(z, lo), hi); }

// Breakpoint of one element, (y - bound)/a with a != 0: the multiplier at
// which the element reaches its bound (Appendix A.1).  The reciprocal of a is
// refined by two Newton steps, so the quotient is within a few ulps of the
// correctly rounded one at a third of the cost of a full division.  Only the
// largest breakpoint is used, as the end of the search bracket (the smallest
// multiplier at which every element is saturated).
__device__ __forceinline__ double recip(double av) {
  double r = __builtin_amdgcn_rcp(av);
  r = fma(r, fma(-av, r, 1.0), r);
  return fma(r, fma(-av, r, 1.0), r);
}
__device__ __forceinline__ double breakpoint(double y, double av, double bound) { return (y - bound) * recip(av); }

// ------------------------------------------------------------------ cross-workgroup publication
// Values one workgroup writes for another (per-tile partial sums, the pass
// totals) are stored with agent-coherent stores, which write through this
// XCD's L2 to memory, and read with agent-coherent loads, which do not hit a
// stale line in the reader's L2.  Every wave that stores such values waits
// for its own stores to complete before the workgroup barrier that precedes
// the flag or go word: a barrier orders the waves of one workgroup only, and
// a release by another wave covers that wave's own stores, so without the
// wait a store of wave k could still be in flight when the flag is seen.
// With the data in memory before the flag is raised, flags and go words need
// no release fence (no write-back of the whole L2 per workgroup and pass).
__device__ __forceinline__ void publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch_published(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): this wave's
// vector memory operations, stores included, have completed.
__device__ __forceinline__ void wait_own_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce NV per-thread values over the workgroup and store them as the
// partials of `tile` (value-major layout).  Values whose bit is set in
// `maxmask` are maxima, the rest sums.  Fixed order: the values go through
// LDS in chunks of 8; wave w reduces value c + w of chunk c, each lane first
// summing 8 threads' entries in a fixed order, then an xor butterfly.
template <int NV>
__device__ __forceinline__ void block_to_part(const double (&acc)[NV], int nv, uint64_t maxmask,
                                              double* red, double* pb, int tile) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int c = 0; c < NV; c += NWAVE) {
#pragma unroll
    for (int j = 0; j < NWAVE; ++j)
      if (c + j < NV) red[j * BLOCK + tid] = acc[c + j];
    __syncthreads();
    const int v = c + w;
    if (v < nv) {
      const bool mx = v < 64 && ((maxmask >> v) & 1);
      const double* col = red + w * BLOCK;
      double r = col[lane];
#pragma unroll
      for (int k = 1; k < BLOCK / 64; ++k) {
        const double q = col[k * 64 + lane];
        r = mx ? fmax(r, q) : r + q;
      }
      r = mx ? wave_max(r) : wave_sum(r);
      if (lane == 0) publish(&pb[v * TILES_PAD + tile], r);
    }
    // no wait for the stores here: a workgroup reduces many tiles per pass
    // and a wait would drain its loads and stores at every tile; the grid
    // barrier waits for them once, before the pass's flag
    __syncthreads();
  }
}

// Reduce the per-tile partials of every segment: tot[s * nv + v].  Every
// workgroup runs this on the same data in the same order.
__device__ __forceinline__ void reduce_tiles(const double* pb, int nv, uint64_t maxmask, const int32_t* tile_base,
                             int nseg, double* tot) {
  constexpr int LMAX = 8;               // loads in flight per thread
  const int pairs = nseg * nv;
  int P = 64;
  while (P > 1 && pairs * P > BLOCK) P >>= 1;
  const int total = pairs * P;
  for (int base = 0; base < total; base += BLOCK) {
    const int idx = base + threadIdx.x;
    const int pair = idx / P, g = idx % P;
    const bool act = pair < pairs;
    int v = 0, s = 0;
    if (act) { s = pair / nv; v = pair % nv; }
    const bool mx = act && v < 64 && ((maxmask >> v) & 1);
    double r = mx ? -INFINITY : 0.0;
    if (act) {
      const int te = tile_base[s + 1];
      for (int t0 = tile_base[s] + g; t0 < te; t0 += LMAX * P) {
        double q[LMAX];
#pragma unroll
        for (int k = 0; k < LMAX; ++k) {
          const int t = t0 + k * P;
          q[k] = (t < te) ? fetch_published(&pb[v * TILES_PAD + t]) : (mx ? -INFINITY : 0.0);
        }
#pragma unroll
        for (int k = 0; k < LMAX; ++k) r = mx ? fmax(r, q[k]) : r + q[k];
      }
    }
    for (int o = P >> 1; o > 0; o >>= 1) {
      const double q = __shfl_xor(r, o, 64);
      r = mx ? fmax(r, q) : r + q;
    }
    if (act && g == 0) tot[s * nv + v] = r;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ tracing

__device__ __forceinline__ uint64_t clk() { return __builtin_amdgcn_s_memrealtime(); }

// This workgroup's index among the workgroups that solve the instance, and
// their number (a one-instance launch: blockIdx.x and gridDim.x; a server
// slot: its own range of the grid).
__device__ __forceinline__ int wg_id(const Desc& d) { return (int)blockIdx.x - d.wg_base; }
__device__ __forceinline__ int wg_num(const Desc& d) { return d.wg_count; }

__device__ __forceinline__ void trace_put(const Desc& d, int pass, int slot, uint64_t v) {
  if (d.trace && wg_id(d) == 0 && threadIdx.x == 0 && pass < TRACE_MAX) d.trace[pass * TRACE_W + slot] = v;
}
// per-workgroup records of each pass, after the per-pass records: loop start,
// loop end, go seen (end of the pass's wait), hardware ids (HW_ID | XCC_ID << 32)
__device__ __forceinline__ uint64_t* trace_wg_rec(const Desc& d, int pass) {
  return d.trace + TRACE_MAX * TRACE_W + ((size_t)pass * GMAX + wg_id(d)) * TRACE_WG_W;
}
__device__ __forceinline__ void trace_wg(const Desc& d, int pass, uint64_t t_start, uint64_t t_end) {
  if (d.trace && threadIdx.x == 0 && pass < TRACE_WG_PASSES) {
    uint64_t* r = trace_wg_rec(d, pass);
    r[0] = t_start;
    r[1] = t_end;
    // HW_ID (hwreg 4, all 32 bits) and XCC_ID (hwreg 20, low 4 bits)
    const uint32_t hw = __builtin_amdgcn_s_getreg(4 | (0 << 6) | (31 << 11));
    const uint32_t xcc = __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11));
    r[3] = (uint64_t)hw | ((uint64_t)xcc << 32);
  }
}
__device__ __forceinline__ void trace_wg_go(const Desc& d, int pass, uint64_t t) {
  if (d.trace && threadIdx.x == 0 && pass < TRACE_WG_PASSES) trace_wg_rec(d, pass)[2] = t;
}
// records of the last workgroup (slots 6, 7)
__device__ __forceinline__ void trace_last(const Desc& d, int pass, int slot, uint64_t v) {
  if (d.trace && wg_id(d) == wg_num(d) - 1 && threadIdx.x == 0 && pass < TRACE_MAX) d.trace[pass * TRACE_W + slot] = v;
}

// ------------------------------------------------------------------ grid synchronisation

// One pass ends with every workgroup publishing a launch-unique epoch on its
// own cache line (no shared counter: device-scope atomics on one address
// serialise at the memory side and cost ~G x 70 ns).  Workgroup 0 waits for
// all flags with all its threads, reduces the per-tile partials once (fixed
// order), and publishes the totals and a go word in NREP copies 1 KiB apart;
// every other workgroup polls and reads only its own copy, so that no single
// line is polled by hundreds of workgroups (that queues the polls at one
// memory channel and staggers the start of the next pass by microseconds).
// Every wait is bounded: on expiry the error word records this launch's epoch
// and every workgroup leaves.
constexpr int FLAG_STRIDE = 16;     // uint64 per flag: one 128-byte line each
constexpr int REP_VALS = REP_WORDS - 1;

struct SyncWords {
  uint64_t* flags;   // [GMAX * FLAG_STRIDE]
  uint64_t* rep;     // [NREP * REP_WORDS]: go word, then totals (double) when they fit
  uint64_t* err;     // one line: epoch of the launch that timed out
  double* totals;    // [TOT_MAX], used when the totals do not fit a copy
};

__device__ __forceinline__ SyncWords sync_words(const Desc& d) {
  SyncWords w;
  w.flags = d.sync;
  w.rep = d.sync + (size_t)GMAX * FLAG_STRIDE;
  w.err = w.rep + (size_t)NREP * REP_WORDS;
  w.totals = (double*)(w.err + FLAG_STRIDE);
  return w;
}

__device__ __forceinline__ bool grid_reduce(const Desc& d, uint64_t epoch, const double* pb, int nv, uint64_t maxmask,
                            int nseg, double* tot, int32_t* abort_flag, int pass_no) {
  const SyncWords W = sync_words(d);
  const int G = wg_num(d);
  const int wid = wg_id(d);
  const int ntot = nseg * nv;
  const bool in_rep = ntot <= REP_VALS;
  // every wave's stores of this pass (tile partials, streamed outputs) are
  // complete before the barrier that precedes the flag
  wait_own_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    *abort_flag = 0;
    // the partials of every wave are in memory
    __hip_atomic_store(&W.flags[(size_t)wid * FLAG_STRIDE], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (d.allred) {
    // every workgroup waits for every flag, then reduces the partials itself
    // in the same fixed order (so every workgroup holds the same bits); a
    // workgroup writes this buffer again two passes later, after every
    // workgroup has raised the next pass's flag, which it does only after
    // this read
    bool ok = true;
    for (int w = threadIdx.x; w < G && ok; w += BLOCK) {
      uint32_t spins = 0;
      while (__hip_atomic_load(&W.flags[(size_t)w * FLAG_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT || __hip_atomic_load(W.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == d.epoch0) {
          ok = false;
          break;
        }
      }
    }
    if (!ok) atomicOr(abort_flag, 1);
    __syncthreads();
    if (*abort_flag) {
      if (threadIdx.x == 0) __hip_atomic_store(W.err, d.epoch0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    trace_put(d, pass_no, 2, clk());
    trace_wg_go(d, pass_no, clk());
    reduce_tiles(pb, nv, maxmask, d.tile_base, nseg, tot);
    trace_put(d, pass_no, 3, clk());
    return true;
  }
  if (wid == 0) {
    bool ok = true;
    for (int w = threadIdx.x; w < G && ok; w += BLOCK) {
      uint32_t spins = 0;
      while (__hip_atomic_load(&W.flags[(size_t)w * FLAG_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT) { ok = false; break; }
      }
    }
    if (!ok) atomicOr(abort_flag, 1);
    __syncthreads();
    // the partials are read with agent-coherent loads (no acquire fence, which
    // would invalidate this XCD's whole L2)
    if (threadIdx.x == 0 && *abort_flag) __hip_atomic_store(W.err, d.epoch0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (*abort_flag) return false;
    trace_put(d, pass_no, 2, clk());
    reduce_tiles(pb, nv, maxmask, d.tile_base, nseg, tot);
    trace_put(d, pass_no, 3, clk());
    if (in_rep) {
      for (int i = threadIdx.x; i < NREP * ntot; i += BLOCK) {
        const int r = i / ntot, k = i - r * ntot;
        publish((double*)(W.rep + (size_t)r * REP_WORDS + 1) + k, tot[k]);
      }
    } else {
      for (int i = threadIdx.x; i < ntot; i += BLOCK) publish(W.totals + i, tot[i]);
    }
    wait_own_stores();
    __syncthreads();
    // one wave raises every copy of the go word; the totals of every wave are in memory
    if (threadIdx.x < 64) {
      for (int r = threadIdx.x; r < NREP; r += 64)
        __hip_atomic_store(W.rep + (size_t)r * REP_WORDS, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
  }
  trace_last(d, pass_no, 6, clk());
  uint64_t* my = W.rep + (size_t)(wid % NREP) * REP_WORDS;
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    bool ok = true;
    while (__hip_atomic_load(my, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT || __hip_atomic_load(W.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == d.epoch0) {
        ok = false;
        break;
      }
    }
    if (!ok) {
      __hip_atomic_store(W.err, d.epoch0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *abort_flag = 1;
    }
  }
  __syncthreads();
  if (*abort_flag) return false;
  trace_last(d, pass_no, 7, clk());
  trace_wg_go(d, pass_no, clk());
  // The totals are the only data of other workgroups read here: device-scope
  // loads of them, issued after the go word was seen, return what workgroup 0
  // wrote back before raising it.  No acquire fence: it would invalidate this
  // XCD's whole L2 once per workgroup and pass.
  uint64_t* src = in_rep ? my + 1 : (uint64_t*)W.totals;
  for (int i = threadIdx.x; i < ntot; i += BLOCK)
    tot[i] = __builtin_bit_cast(double, __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  __syncthreads();
  return true;
}

// Workgroup 0 reports a timeout of this launch in the result.
__device__ __forceinline__ void report_error(const Desc& d, int32_t* err_field) {
  if (wg_id(d) == 0 && threadIdx.x == 0 && err_field) {
    const SyncWords W = sync_words(d);
    if (__hip_atomic_load(W.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == d.epoch0)
      *err_field = PGDTO_ERR_TIMEOUT;
  }
}

// ------------------------------------------------------------------ descriptor in LDS

// The launch descriptor is the kernel's only argument.  Each workgroup copies
// it once from the kernarg segment into LDS and reads it from there; naming
// the by-value parameter would make the compiler copy it to private memory
// for every lane.
__device__ __forceinline__ void load_desc(Desc& sd) {
  const uint32_t* src = (const uint32_t*)__builtin_amdgcn_kernarg_segment_ptr();
  uint32_t* dst = reinterpret_cast<uint32_t*>(&sd);
  for (int i = threadIdx.x; i < (int)(sizeof(Desc) / 4); i += BLOCK) dst[i] = src[i];
  __syncthreads();
}

// ------------------------------------------------------------------ tile geometry

struct TileGeom {
  int seg;
  int64_t sstart, send;   // segment bounds (valid elements)
  int64_t ts, te;         // tile element range (ts 32-aligned)
  int64_t p0;             // first vector slot of the tile
  int nsweep;             // vector slots per thread (uniform over the block)
  bool interior;          // a whole tile inside its segment: every slot full, nsweep even
};

template <typename T>
__device__ __forceinline__ TileGeom tile_geom(const Desc& d, int tile) {
  constexpr int V = VT<T>::N;
  TileGeom g;
  int s = 0;
  while (s + 1 < d.nseg && d.tile_base[s + 1] <= tile) ++s;
  g.seg = s;
  g.sstart = d.off[s];
  g.send = d.off[s + 1];
  const int64_t astart = g.sstart & ~(int64_t)31;      // 32-element aligned (free-mask words)
  const int64_t ts = astart + (int64_t)(tile - d.tile_base[s]) * d.tile_elems;
  const int64_t te = min(ts + d.tile_elems, g.send);
  g.ts = ts;
  g.te = te;
  g.p0 = ts / V;
  const int64_t nslots = (te - ts + V - 1) / V;
  g.nsweep = (int)((nslots + BLOCK - 1) / BLOCK);
  // tile_elems is a multiple of 2 * BLOCK * V, so a whole tile has an even
  // number of full slots per thread
  g.interior = ts >= g.sstart && ts + d.tile_elems <= g.send;
  return g;
}

// For slot index k of this thread: element base e0, whether the whole vector
// is valid, and the validity mask.
template <typename T>
__device__ __forceinline__ bool slot(const TileGeom& g, int k, int64_t& e0, bool& full, uint32_t& mask) {
  constexpr int V = VT<T>::N;
  const int64_t p = g.p0 + (int64_t)k * BLOCK + threadIdx.x;
  e0 = p * V;
  if (e0 >= g.send) { mask = 0; full = false; return false; }
  full = (e0 >= g.sstart) && (e0 + V <= g.send);
  mask = 0;
#pragma unroll
  for (int q = 0; q < V; ++q)
    if (e0 + q >= g.sstart && e0 + q < g.send) mask |= 1u << q;
  return mask != 0;
}

// Stream a tile in chunks of U vector slots per thread: the loads of all U
// slots (NS streams each) are issued before any of them is used, so each
// wave keeps U * NS 16-byte loads in flight.  f(buf, e0, mask, full) gets the
// NS loaded vectors of one slot.
template <typename T, int NS, int U, bool NT = false, class F>
__device__ __forceinline__ void stream_tile(const TileGeom& g, int64_t n, const T* const* ptrs, F&& f) {
  constexpr int V = VT<T>::N;
  static_assert(U == 1 || U == 2 || U == 4, "chunk of 1, 2 or 4 slots");
  if (g.interior) {
    // every slot whole and inside the segment: no per-element masks or
    // address clamps (f sees a constant full mask and folds its checks away)
    constexpr uint32_t FULL = (1u << V) - 1u;
    const int64_t base = (g.p0 + (int64_t)threadIdx.x) * V;
    auto chunk = [&](int k0, auto uc) __attribute__((always_inline)) {
      constexpr int UU = decltype(uc)::value;
      T buf[UU][NS][V];
      int64_t e0[UU];
#pragma unroll
      for (int u = 0; u < UU; ++u) e0[u] = base + (int64_t)(k0 + u) * (BLOCK * V);
#pragma unroll
      for (int u = 0; u < UU; ++u)
#pragma unroll
        for (int q = 0; q < NS; ++q) ld_vec_whole<T, NT>(gptr(ptrs[q]), e0[u], buf[u][q]);
#pragma unroll
      for (int u = 0; u < UU; ++u) f(buf[u], e0[u], FULL, true);
    };
    // nsweep is even here: chunks of U, then at most one chunk of 2
    int k0 = 0;
    if constexpr (NT) {
      // two chunk buffers: the loads of chunk k + 1 are issued before chunk k
      // is used, so each wave keeps loads in flight while it computes (the
      // scheduling barriers stop the compiler from sinking them behind the
      // work).  Stores in f go to the chunk being used, never to the one in
      // flight (outputs alias inputs only index for index).
      const int nfull = g.nsweep / U * U;
      T b0[U][NS][V], b1[U][NS][V];
      auto load = [&](T (&b)[U][NS][V], int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < NS; ++q)
            ld_vec_whole<T, NT>(gptr(ptrs[q]), base + (int64_t)(c0 + u) * (BLOCK * V), b[u][q]);
      };
      auto use = [&](T (&b)[U][NS][V], int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u) f(b[u], base + (int64_t)(c0 + u) * (BLOCK * V), FULL, true);
      };
      if (nfull > 0) load(b0, 0);
      while (k0 < nfull) {
        if (k0 + U < nfull) load(b1, k0 + U);
        __builtin_amdgcn_sched_barrier(0);
        use(b0, k0);
        k0 += U;
        if (k0 >= nfull) break;
        if (k0 + U < nfull) load(b0, k0 + U);
        __builtin_amdgcn_sched_barrier(0);
        use(b1, k0);
        k0 += U;
      }
    } else {
      for (; k0 + U <= g.nsweep; k0 += U) chunk(k0, std::integral_constant<int, U>{});
    }
    if constexpr (U == 4) {
      if (k0 < g.nsweep) chunk(k0, std::integral_constant<int, 2>{});
    }
    return;
  }
  for (int k0 = 0; k0 < g.nsweep; k0 += U) {
    T buf[U][NS][V];
    int64_t e0[U];
    uint32_t mask[U];
    bool full[U], ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = k0 + u < g.nsweep;     // uniform over the block
      ok[u] = live && slot<T>(g, k0 + u, e0[u], full[u], mask[u]);
      if (!live) e0[u] = n;                    // reads zeros
    }
    // every lane loads (a slot past the end reads zeros), so the loads of
    // the whole chunk stay in flight together
    ld_slots<T, U, NS, NT>(ptrs, e0, n, buf);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) f(buf[u], e0[u], mask[u], full[u]);
  }
}

// ------------------------------------------------------------------ 1-D search control

// Per-row bracket state of a 1-D search on phi(lam) = a.x(lam) - b - kappa lam
// (nonincreasing, piecewise linear; Appendix A.1).  lo < root < hi, with
// f = phi at the ends and s = -phi' (sum of a^2 over free elements + kappa).
struct Search {
  double lo[PGDTO_MAX_BLOCKS], hi[PGDTO_MAX_BLOCKS];
  double flo[PGDTO_MAX_BLOCKS], fhi[PGDTO_MAX_BLOCKS];
  double slo[PGDTO_MAX_BLOCKS], shi[PGDTO_MAX_BLOCKS];
  double lam[PGDTO_MAX_BLOCKS], scale[PGDTO_MAX_BLOCKS], width[PGDTO_MAX_BLOCKS];
  double ssat[PGDTO_MAX_BLOCKS];
  double err[PGDTO_MAX_BLOCKS];     // stated |lam - lam*| at exit (before the rounding allowance)
  double slope[PGDTO_MAX_BLOCKS];   // slope of the dual function at exit (0: unknown or flat)
  double trial[PGDTO_MAX_BLOCKS][NT];
  int32_t state[PGDTO_MAX_BLOCKS], outcome[PGDTO_MAX_BLOCKS], npass[PGDTO_MAX_BLOCKS];
  int32_t shrunk[PGDTO_MAX_BLOCKS];
  int32_t cmode[PGDTO_MAX_BLOCKS];  // free-set compaction: 0 not yet, 1 in the coming pass, 2 done
};

__device__ __forceinline__ bool inside(double v, double lo, double hi) { return v > lo && v < hi; }

__device__ __forceinline__ void search_pick(Search& S, int s, int mode, bool lean) {
  const double lo = S.lo[s], hi = S.hi[s];
  const double mid = 0.5 * (lo + hi);
  if (mode == PGDTO_SEARCH_BISECT) {
    S.trial[s][0] = mid;
    S.trial[s][1] = NAN;
    return;
  }
  const double sec = lo + S.flo[s] * ((hi - lo) / (S.flo[s] - S.fhi[s]));
  const double nlo = S.slo[s] > 0.0 ? lo + S.flo[s] / S.slo[s] : NAN;
  const double nhi = S.shi[s] > 0.0 ? hi + S.fhi[s] / S.shi[s] : NAN;
  // First trial: the Newton point from the lower end (the tangent of the
  // piecewise-linear dual there), else the secant, else the midpoint.
  // Second trial: the Newton point from the upper end when the previous
  // pass halved the bracket.  lean (the 1-D searches): otherwise, and while
  // the upper end has no slope yet, twice the Newton step from the lower end
  // -- the dual is typically convex there, so the tangent from below
  // undershoots and the doubled step brackets the root from above, which
  // lets the next steps close in from both sides and narrows the bracket
  // early (the free-set compaction below needs a narrow bracket).  Without
  // lean, a pass that did not halve the bracket is followed by a midpoint.
  double t0 = inside(nlo, lo, hi) ? nlo : (inside(sec, lo, hi) ? sec : mid);
  if (!inside(t0, lo, hi)) t0 = mid;
  const double ext = lo + 2.0 * (nlo - lo);
  const bool doubled = lean && inside(nlo, lo, hi) && inside(ext, lo, hi);
  double t1;
  // a bracket that did not halve: the doubled Newton step from below (the
  // distance covered from below at least doubles every pass), else the
  // midpoint (the bracket halves)
  if (!S.shrunk[s]) t1 = doubled ? ext : mid;
  else if (inside(nhi, lo, hi) && nhi != t0) t1 = nhi;
  else if (lean && inside(nlo, lo, hi) && inside(ext, lo, hi)) t1 = ext;
  else if (inside(sec, lo, hi) && sec != t0) t1 = sec;
  else t1 = mid;
  if (t1 == t0 || !inside(t1, lo, hi)) t1 = NAN;
  S.trial[s][0] = t0;
  S.trial[s][1] = t1;
}

// Initialise row/block s from the lam = 0 pass.  Returns true if the search
// must run.  f0 = phi(0); s0 = -phi'(0); bp = largest breakpoint (the end of
// Alg. 1's bracket, -y_l); ssat = a.x over the saturated point.
__device__ __forceinline__ bool search_init(Search& S, int s, double f0, double s0, double bp, double ssat,
                            double b, double kappa, double scale, int mode, bool lean) {
  S.npass[s] = 0;
  S.width[s] = 0.0;
  S.scale[s] = scale;
  S.ssat[s] = ssat;
  S.shrunk[s] = 1;
  S.err[s] = 0.0;                     // the exits below are exact up to rounding
  S.slope[s] = s0;
  if (!(f0 > 0.0)) {                  // delta(0) feasible: y* = 0 (Alg. 1, first branch)
    S.lam[s] = 0.0;
    S.outcome[s] = PGDTO_INACTIVE;
    S.state[s] = SEG_DONE;
    return false;
  }
  if (!(bp > 0.0) || !isfinite(bp)) bp = 0.0;
  const double fhi = ssat - b - kappa * bp;
  if (fhi >= 0.0) {
    // no sign change inside the bracket: every element with a_i != 0 is
    // saturated from bp on; phi is linear there with slope -kappa.
    S.slope[s] = kappa;
    if (kappa > 0.0) {
      S.lam[s] = bp + fhi / kappa;
      S.outcome[s] = (ssat - b > 0.0) ? PGDTO_INFEASIBLE : PGDTO_CONVERGED;
    } else {
      S.lam[s] = bp;
      S.outcome[s] = (fhi > 0.0) ? PGDTO_INFEASIBLE : PGDTO_CONVERGED;
    }
    S.state[s] = SEG_DONE;
    return false;
  }
  S.lo[s] = 0.0; S.flo[s] = f0; S.slo[s] = s0;
  S.hi[s] = bp;  S.fhi[s] = fhi; S.shi[s] = kappa;
  S.state[s] = SEG_SEARCH;
  search_pick(S, s, mode, lean);
  return true;
}

// Warm start: the first pass evaluates lam0 (when inside the bracket) and
// the cold first trial as its second trial.  A lam0 within the stop
// tolerance ends the search in that pass; otherwise the bracket update keeps
// whichever of the two ends up closer, and the search goes on from there.
__device__ __forceinline__ void search_warm(Search& S, int s, double lam0) {
  if (!inside(lam0, S.lo[s], S.hi[s])) return;
  const double t0 = S.trial[s][0];
  S.trial[s][0] = lam0;
  S.trial[s][1] = (t0 == lam0) ? NAN : t0;
}

// Update row/block s from the sums of one search pass.  fsum[t] = a.x(trial_t),
// ssum[t] = sum over free elements of a^2 at trial_t.
__device__ __forceinline__ void search_update(Search& S, int s, double f0sum, double f1sum, double s0sum, double s1sum,
                              double b, double kappa, double tol_n, double tol_b, int max_pass, int mode,
                              bool lean) {
  const double fsum[NT] = {f0sum, f1sum};
  const double ssum[NT] = {s0sum, s1sum};
  const double eps = tol_n * S.scale[s];
  const double w0 = S.hi[s] - S.lo[s];
  double best = NAN, bestf = INFINITY, bests = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double lt = S.trial[s][t];
    if (!(lt == lt)) continue;
    const double f = fsum[t] - b - kappa * lt;
    const double sl = ssum[t] + kappa;
    if (mode != PGDTO_SEARCH_BISECT && fabs(f) <= eps && fabs(f) < bestf) { best = lt; bestf = fabs(f); bests = sl; }
    if (f > 0.0 && lt > S.lo[s]) { S.lo[s] = lt; S.flo[s] = f; S.slo[s] = sl; }
    else if (f <= 0.0 && lt < S.hi[s]) { S.hi[s] = lt; S.fhi[s] = f; S.shi[s] = sl; }
  }
  S.npass[s] += 1;
  const double lo = S.lo[s], hi = S.hi[s];
  const double w = hi - lo;
  S.shrunk[s] = (w <= 0.5 * w0) ? 1 : 0;
  if (best == best) {
    // the root lies in the bracket, of which `best` is an end; on the
    // linear piece through `best` it is |f| / slope away (twice that stated)
    S.lam[s] = best;
    S.width[s] = w;
    S.slope[s] = bests;
    S.err[s] = (bestf == 0.0) ? 0.0 : (bests > 0.0 ? fmin(w, 2.0 * bestf / bests) : w);
    S.outcome[s] = PGDTO_CONVERGED;
    S.state[s] = SEG_DONE;
    return;
  }
  const double res = 4.0 * fmax(fabs(hi), 1e-300) * 2.220446049250313e-16;
  const double wtol = (mode == PGDTO_SEARCH_BISECT) ? fmax(tol_b, res) : res;
  if (w <= wtol || S.fhi[s] == 0.0 || S.npass[s] >= max_pass) {
    // the linear interpolation of the bracket is exact when no breakpoint lies inside
    double l = (S.fhi[s] == 0.0) ? hi : lo + S.flo[s] * (w / (S.flo[s] - S.fhi[s]));
    if (!(l >= lo && l <= hi)) l = 0.5 * (lo + hi);
    S.lam[s] = l;
    S.width[s] = w;
    S.slope[s] = (S.fhi[s] == 0.0) ? S.shi[s] : 0.5 * (S.slo[s] + S.shi[s]);
    S.err[s] = (S.fhi[s] == 0.0) ? 0.0 : w;
    S.outcome[s] = (S.npass[s] >= max_pass && w > wtol && S.fhi[s] != 0.0) ? PGDTO_MAXITER : PGDTO_CONVERGED;
    S.state[s] = SEG_DONE;
    return;
  }
  search_pick(S, s, mode, lean);
}

// Automatic penalty (Appendix A.2): with tau the tolerated constraint
// violation, C = 2 bp / tau, i.e. kappa = tau / bp, bp the largest breakpoint
// over the rows (the end of every row's bracket).  Rows with a non-finite or
// non-positive breakpoint do not count; with none left kappa = 0.
__device__ __forceinline__ double auto_kappa(double tau, const double* bp, int stride, int rows) {
  double mx = 0.0;
  for (int j = 0; j < rows; ++j) {
    const double v = bp[j * stride];
    if (isfinite(v) && v > mx) mx = v;
  }
  return mx > 0.0 ? tau / mx : 0.0;
}

// Stated error of a multiplier: the estimate `est` of |lam - lam*| plus 16
// float64 rounding units of |lam| and of sigma / slope (the shift of the root
// that a rounding-level error of the sums moves it by); a zero slope (a flat
// stretch of the dual at kappa = 0, where lam is not unique) states INFINITY
// unless the estimate is exact.
__device__ __forceinline__ double lam_error(double lam, double est, double sigma, double slope) {
  constexpr double U16 = 16.0 * 2.220446049250313e-16;
  if (!(est == est)) return INFINITY;
  if (!(slope > 0.0)) return (est == 0.0) ? U16 * fabs(lam) : INFINITY;
  return est + U16 * (fabs(lam) + sigma / slope);
}

// Half a unit in the last place of the stream dtype at v >= 0: the rounding
// of a value of magnitude at most v when x is stored.
__device__ __forceinline__ double half_ulp(double v, bool f32) {
  int e = 0;
  (void)frexp(v, &e);                   // v = f 2^e, f in [0.5, 1)
  return ldexp(1.0, e - (f32 ? 25 : 54));
}

// Control parameters, copied once into LDS so that no reference to the
// kernel argument escapes into out-of-line functions (it would be copied to
// private memory per lane).
struct CtlParams {
  double kappa, tol_n, tol_b, c1, c2;
  int32_t max_newton, max_ls, max_search, ncp, search, eq;   // eq: equality-row bits
};

__device__ __forceinline__ void load_ctl(const Desc& d, CtlParams& P) {
  P.kappa = d.kappa; P.tol_n = d.tol_n; P.tol_b = d.tol_b; P.c1 = d.c1; P.c2 = d.c2;
  P.max_newton = d.max_newton; P.max_ls = d.max_ls; P.max_search = d.max_search;
  P.ncp = d.ncp; P.search = d.search; P.eq = (int32_t)(d.eq_mask & 0xffu);
}

__device__ __forceinline__ int severity(int o) {
  switch (o) {
    case PGDTO_INACTIVE: return 0;
    case PGDTO_CONVERGED: return 1;
    case PGDTO_INFEASIBLE: return 2;
    case PGDTO_MAXITER: return 3;
    default: return 4;
  }
}

// ------------------------------------------------------------------ Alg. 3 step rule

struct PgdScalars {
  double alpha, beta;
  int32_t used_fb;
};

// Step size of Alg. 3 (fallback at t = 0 and, after warm-up, on constraint
// violation; otherwise eq. final_alpha with eps_alpha) and beta of eq. CG.
// v: ss, yy, sy, gg, gdg (= grad.(grad - grad_prev)), gpgp, ginf.
__device__ __forceinline__ void pgd_scalars(const Desc& d, const double* v, PgdScalars& o) {
  const double ss = v[0], yy = v[1], sy = v[2], gg = v[3], gdg = v[4], gpgp = v[5], ginf = v[6];
  const double fb = (ginf > 0.0) ? fmin(d.alpha_max, d.alpha_fallback / ginf) : d.alpha_max;
  o.used_fb = 0;
  if (d.fallback_forced || yy == 0.0) {
    o.alpha = fb;
    o.used_fb = 1;
  } else {
    const double lip = sqrt(ss) / sqrt(yy);
    o.alpha = (sy > d.eps_alpha) ? fmin(fmin(ss / sy, 2.0 * lip), d.alpha_max) : fmin(lip, d.alpha_max);
  }
  double beta = 0.0;
  if (!d.zero_step && d.cg_rule != PGDTO_CG_NONE && gpgp > 0.0) {
    beta = (d.cg_rule == PGDTO_CG_FR) ? gg / gpgp : fmax(gdg / gpgp, 0.0);
  }
  o.beta = beta;
}


// ------------------------------------------------------------------ arrival door
// One-instance launches are ordinary launches (a cooperative launch costs the
// runtime about 17 us more per launch), so that all of the grid is resident
// is not guaranteed; the grid barrier needs every participant running.  Each
// workgroup therefore takes a ticket at entry with one atomic add on the
// context's door word, [generation:32 | closed:1 | count:31].  The first
// arrival waits (bounded: Desc::door_wait, 30 us by default) until the whole
// grid has arrived, closes the door
// and publishes the count; a workgroup arriving after that leaves at once,
// and the participants take their ticket as workgroup id.  Results do not
// depend on the count (tile-ordered reductions).  The last of the grid's
// arrivals (the first one when nobody came late) reopens the door with the
// next generation, and the generation also gives the launch's barrier epochs:
// nothing the host wrote for this launch has to be unique, so a replayed
// graph of launches works as the launches did.
constexpr uint64_t DOOR_CLOSED = 1ull << 31;
constexpr uint64_t DOOR_COUNT = DOOR_CLOSED - 1;

__device__ __forceinline__ uint64_t* door_words(const Desc& d) {
  return d.sync + (size_t)GMAX * FLAG_STRIDE + (size_t)NREP * REP_WORDS + FLAG_STRIDE + TOT_MAX;
}

// false: this workgroup arrived after the door closed and must leave.
__device__ __forceinline__ bool enter_launch(Desc& sd, int32_t* late_sh) {
  if (threadIdx.x == 0) {
    uint64_t* door = door_words(sd);
    uint64_t* pub = door + FLAG_STRIDE;      // [generation + 1 : 32 | count : 32]
    const uint64_t G = gridDim.x;
    const uint64_t old = __hip_atomic_fetch_add(door, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t gen = old >> 32;
    const uint64_t next_open = (gen + 1) << 32;
    int late = (old & DOOR_CLOSED) != 0;
    const uint64_t ticket = old & DOOR_COUNT;
    uint64_t count = 0;
    if (late) {
      if (ticket == G - 1)                   // the grid's last arrival: reopen for the next launch
        __hip_atomic_store(door, next_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (ticket == 0) {
      const uint64_t t0 = clk();
      while ((__hip_atomic_load(door, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & DOOR_COUNT) < G &&
             clk() - t0 < sd.door_wait)
        __builtin_amdgcn_s_sleep(1);
      const uint64_t fin = __hip_atomic_fetch_or(door, DOOR_CLOSED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      count = fin & DOOR_COUNT;
      // the whole grid is in: no one else touches this launch's door
      if (count == G) __hip_atomic_store(door, next_open, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(pub, ((gen + 1) << 32) | count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // the first arrival is running and publishes within the wait above;
      // the spin cap only guards against the impossible
      uint64_t v = 0;
      uint32_t spins = 0;
      while (((v = __hip_atomic_load(pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != gen + 1) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT) break;
      }
      if ((v >> 32) == gen + 1) count = v & 0xffffffffull;
      else late = 1;
    }
    if (!late) {
      sd.wg_base = (int32_t)blockIdx.x - (int32_t)ticket;
      sd.wg_count = (int32_t)count;
      // barrier epochs of this launch: above every flag an earlier launch of
      // this context left (generations grow by one per launch)
      sd.epoch0 = (gen + 1) << 20;
    }
    *late_sh = late;
  }
  __syncthreads();
  return *late_sh == 0;
}

}  // namespace pgdto
