// Projection kernels for gfx950 (CDNA4, wave64).
//
// One persistent launch solves a whole projection: every pass
// streams y (and the constraint rows) once, each workgroup reduces its tiles
// into per-tile partial sums and publishes an epoch flag; workgroup 0 sums
// the per-tile partials in a fixed order and broadcasts the totals; then
// EVERY workgroup runs the same float64 control logic (bracket update,
// Newton step, line search) on bit-identical totals, so all workgroups agree
// on the next pass without the host.
//
// Paper references: x(lam) = clip(y - A^T lam) (Theorems 1/2, eq. delta_y),
// h (eq. h), J = A D A^T + kappa I (eq. reg_jacobian), Algorithm 1 (bracket
// search on the monotone dual function of Appendix A.1), Algorithm 2 (Stage 1
// single-active candidates, semismooth Newton with line search, Appendix
// A.2), Algorithm 3 (step size eq. final_alpha, direction eq. CG).
//
// Precision: streams are float32 or float64 in HBM; per-element arithmetic
// is float64 (float64 vector FMA runs at the rate of unpacked float32 on
// CDNA4), sums are float64 per thread, then a fixed LDS/wave tree, then a
// fixed-order cross-tile sum.  The one exception is the free-slope sum of the
// 1-D search with float streams, which only steers the choice of trial points
// and is summed in float.


#include "pgdto_device.h"

#include <mutex>

namespace pgdto {

// ------------------------------------------------------------------ free-set compaction
// Once a row's bracket [bl, bh] is narrow, an element whose state (below,
// inside or above the box) is the same at both ends keeps that state for
// every later trial multiplier in the bracket (z = y - lam a is monotone in
// lam, and so is its correctly rounded fma): its term of a.x(lam) is a
// constant (a lo, a hi) or linear in lam (a y - lam a^2).  The compaction
// pass folds those into per-tile sums S0 (the constants and a y) and Q
// (a^2 of the free ones) and copies the other ("undecided") elements' (y, a)
// pairs to scratch; later passes of the tile then evaluate
//   a.x(lam) = S0 - lam Q + sum over the undecided pairs,
//   slope     = Q + sum of a^2 over the undecided pairs that are free,
// reading a few percent of the bytes.  Only whole interior tiles take part,
// and whether a tile is compacted depends on its data alone (not on the
// workgroups or the route), so every route still gives the same bits.
// Each wave compacts its own share of the tile (tile_elems / NWAVE elements,
// so at most half as many pairs fit its region of the scratch), with a
// wave-level scan and no workgroup barrier; a later pass reduces a
// compacted tile with one wave, so a workgroup evaluates up to NWAVE of its
// compacted tiles at once, each in one round trip to memory.  Per-tile
// metadata sits in rows of the partial-sum table that the 1-D passes do not
// use: per wave, the pairs kept (or -1 when its region overflowed, which
// keeps the tile whole), the folded constant terms S0 and the folded slope Q.
constexpr int META_ROWS = 3 * NWAVE;
constexpr int META_ROW = VMAX - META_ROWS;
constexpr int NV_SEARCH = 2 * NT + 1;      // per trial a.x and slope, then the pairs kept
constexpr int NV_FINAL1 = 5;               // a.x, free count, |x - rho|^2, |x|^2 (pgd), |x - y|^2

__device__ __forceinline__ double* meta_row(const Desc& d, int r) {
  return d.part + (size_t)(META_ROW + r) * TILES_PAD;      // buffer 0
}

// Element state at multiplier lam: 0 below the box, 1 inside, 2 above.
__device__ __forceinline__ int elem_state(double yq, double av, double lam, double lo, double hi) {
  const double z = fma(-lam, av, yq);
  return z < lo ? 0 : (z > hi ? 2 : 1);
}

// A kept (y, a) pair.  Only the workgroup that owns the tile writes and
// later reads it (the tile-to-workgroup map is fixed for a launch), on the
// same CU: plain stores and loads, one 8- or 16-byte access per pair.
template <typename T>
__device__ __forceinline__ void put_pair(T* dst, int64_t j, T y, T a) {
  typedef T P2 __attribute__((ext_vector_type(2)));
  *reinterpret_cast<__attribute__((address_space(1))) P2*>(gptr_w(dst) + 2 * j) = P2{y, a};
}
template <typename T>
__device__ __forceinline__ void get_pair(const T* src, int64_t j, T& y, T& a) {
  typedef T P2 __attribute__((ext_vector_type(2)));
  const P2 v = *reinterpret_cast<const __attribute__((address_space(1))) P2*>(gptr(src) + 2 * j);
  y = v.x;
  a = v.y;
}

// One vector slot per lane, called by every lane of the wave together: the
// slot's undecided elements (bits of ub) are appended at the wave's running
// count `run` in (lane, element) order; `ok` turns false for the wave when
// its capacity `capw` would be exceeded.
template <typename T>
__device__ __forceinline__ void compact_slot(const T* yv, const T* av, uint32_t ub, T* dst, int64_t capw,
                                             int64_t& run, bool& ok) {
  constexpr int V = VT<T>::N;
  const int lane = threadIdx.x & 63;
  const int c = __popc(ub);
  int incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const int total = __shfl(incl, 63, 64);
  if (ok && run + total <= capw) {
    int64_t pos = run + (incl - c);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if ((ub >> q) & 1u) put_pair<T>(dst, pos++, yv[q], av[q]);
    }
  }
  if (run + total > capw) ok = false;
  run += total;
}

// ================================================================== 1-D kernel
// SINGLE and INDEPENDENT: one bracket search per segment, all segments in
// lockstep passes (Alg. 1; Sec. 3.2.2 for independent blocks).

struct Sh1D {
  uint8_t cflag[TILES_PAD];       // per local tile in a search pass: 1 = compacted, evaluated by one wave
  double ncomp[PGDTO_MAX_BLOCKS]; // pairs kept by the compaction per segment (-1: none ran)
  int32_t npc[PGDTO_MAX_BLOCKS];  // search passes that streamed only the kept pairs
  double tot[PGDTO_MAX_BLOCKS * 9];
  double amax[PGDTO_MAX_BLOCKS];  // max_i |a_i| per segment (zero pass)
  double red[NWAVE * BLOCK];
  double bs[PGDTO_MAX_BLOCKS];
  double sg[PGDTO_MAX_BLOCKS];    // -1: an equality row searched in the opposite direction (lam < 0)
  double glob[8];
  Search S;
  PgdScalars pg;
  int32_t phase, abort_flag, passes, pad;
};

// SU: vector slots in flight per stream in the streaming passes.  EQ: the
// instance has rows held at equality (the zero pass adds the opposite
// direction's bracket); CP: the free-set compaction is on.  Separate
// instantiations, so that the common case keeps its register allocation.
template <typename T, bool EQ = false, bool CP = false, int SU = 2, bool NT = false>
__device__ __forceinline__ void solve_1d(Sh1D& sh, const Desc& d, int32_t* buf_end = nullptr) {
  constexpr int V = VT<T>::N;
  constexpr int SU1 = SU > 2 ? SU / 2 : 1;     // for the 3- to 5-stream passes
  const int tid = threadIdx.x;
  const int G = wg_num(d);
  const int wid = wg_id(d);
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  double kappa = d.kappa;           // the automatic penalty replaces it after the zero pass

  if (tid == 0) {
    sh.phase = PH_ZERO;
    sh.abort_flag = 0;
    sh.passes = 0;
    sh.pg.alpha = 0.0; sh.pg.beta = 0.0; sh.pg.used_fb = 0;
  }
  for (int s = tid; s < d.nseg; s += BLOCK) {
    sh.bs[s] = d.b[s];
    sh.sg[s] = 1.0;
    sh.S.state[s] = SEG_DONE; sh.S.lam[s] = 0.0; sh.S.npass[s] = 0; sh.S.width[s] = 0.0;
    sh.S.outcome[s] = PGDTO_INACTIVE; sh.S.scale[s] = 1.0; sh.S.ssat[s] = 0.0;
    sh.S.err[s] = 0.0; sh.S.slope[s] = 0.0; sh.amax[s] = 0.0; sh.S.cmode[s] = 0; sh.ncomp[s] = -1.0; sh.npc[s] = 0;
  }
  __syncthreads();

  int buf = d.buf0 & 1;
  const T* A = (const T*)d.A;
  // CP: the instantiation with the free-set compaction (a request asks for
  // it with compact != 0 and scratch); without it every compaction branch
  // folds away and the kernel keeps the register allocation of the plain search
  T* CB = CP ? (T*)d.cbuf : nullptr;
  T* X = (T*)d.x;
  const T* Y = d.pgd ? (const T*)d.x : (const T*)d.y;

  int pass_no = 0;
  if (d.pgd) {
    // Alg. 3 reductions (pass R), before the main loop so that the resident
    // registers below are not live across it.
    double* pb = d.part + (size_t)buf * VMAX * TILES_PAD;
    const uint64_t t_pass0 = clk();
    trace_put(d, pass_no, 0, ((uint64_t)PH_PGD_R << 56) | (t_pass0 & 0x00ffffffffffffffull));
    const int nv = 8;
    const uint64_t maxmask = 1ull << 6;
    for (int tile = wid; tile < d.ntiles; tile += G) {
      const TileGeom g = tile_geom<T>(d, tile);
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      // s = rho_t - rho_{t-1}, y = grad_t - grad_{t-1}: |s|^2, |y|^2, s.y, |g|^2,
      // g.(g - g_prev), |g_prev|^2, |g|_inf, a.rho_t
      if (d.zero_step) {
        const T* ptr[3] = {(const T*)d.rho, (const T*)d.grad, A};
        stream_tile<T, 3, SU1, NT>(g, d.n, ptr, [&](const T (&b)[3][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            const double r = f64(b[0][q]), gr = f64(b[1][q]), av = f64(b[2][q]);
            acc[3] = fma(gr, gr, acc[3]);
            acc[6] = fmax(acc[6], fabs(gr));
            acc[7] = fma(av, r, acc[7]);
          }
        });
      } else {
        const T* ptr[5] = {(const T*)d.rho, (const T*)d.grad, A, (const T*)d.rho_prev, (const T*)d.grad_prev};
        stream_tile<T, 5, SU1, NT>(g, d.n, ptr, [&](const T (&b)[5][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            const double r = f64(b[0][q]), gr = f64(b[1][q]), av = f64(b[2][q]);
            const double sv = r - f64(b[3][q]), gp = f64(b[4][q]), yv = gr - gp;
            acc[0] = fma(sv, sv, acc[0]);
            acc[1] = fma(yv, yv, acc[1]);
            acc[2] = fma(sv, yv, acc[2]);
            acc[3] = fma(gr, gr, acc[3]);
            acc[4] = fma(gr, yv, acc[4]);
            acc[5] = fma(gp, gp, acc[5]);
            acc[6] = fmax(acc[6], fabs(gr));
            acc[7] = fma(av, r, acc[7]);
          }
        });
      }
      block_to_part<8>(acc, nv, maxmask, sh.red, pb, tile);
    }
    trace_put(d, pass_no, 1, clk());
    trace_wg(d, pass_no, t_pass0, clk());
    if (grid_reduce(d, d.epoch0 + (uint64_t)pass_no + 1, pb, nv, maxmask, d.nseg, sh.tot, &sh.abort_flag, pass_no)) {
      if (tid == 0) {
        double v[7] = {0, 0, 0, 0, 0, 0, -INFINITY};
        for (int s = 0; s < d.nseg; ++s) {
          for (int q = 0; q < 6; ++q) v[q] += sh.tot[s * 8 + q];
          v[6] = fmax(v[6], sh.tot[s * 8 + 6]);
        }
        pgd_scalars(d, v, sh.pg);
        sh.passes += 1;
      }
      for (int s = tid; s < d.nseg; s += BLOCK) sh.bs[s] = d.b[s] + sh.tot[s * 8 + 7];
      __syncthreads();
      if (tid == 0) sh.phase = PH_ZERO;
      trace_put(d, pass_no, 5, clk());
    } else {
      if (tid == 0) sh.phase = PH_DONE;
    }
    __syncthreads();
    ++pass_no;
    buf ^= 1;
  }

  // Register residency: the first tile of this workgroup keeps its y (pgd:
  // rho~) and a slots in registers across passes when it has at most RS
  // vector slots per thread; later passes then read no memory for it.  The
  // batch's streaming variant (NT) keeps none: there a workgroup owns about
  // 16 tiles, residency would save 1/16 of the search reads, and the 64
  // registers it holds through every pass cost more (a 16-instance pgd_step
  // launch ran 1.1% faster without it).  A resident and a streamed tile give
  // the same bits.
  constexpr int RS = NT ? 1 : 8;
  T ry[RS][V], ra[RS][V];
  bool resident = false;
  uint32_t rbits = 0u;      // element-validity masks of the resident slots, V bits each
  // slot geometry of resident slot k
  auto rslot = [&](const TileGeom& g, int k, int64_t& e0, bool& full, uint32_t& mask) __attribute__((always_inline)) {
    e0 = 0; full = false; mask = 0u;
    if (k < g.nsweep) slot<T>(g, k, e0, full, mask);
  };
  auto rmask = [&](int k) __attribute__((always_inline)) -> uint32_t { return (rbits >> (k * V)) & ((1u << V) - 1u); };

  // free-mask bits of one vector slot: 32 / V lanes form one 32-bit word
  auto put_mask = [&](bool any, int64_t e0, uint32_t bits, const TileGeom& g) __attribute__((always_inline)) {
    constexpr int LPW = 32 / V;
    uint32_t w = any ? (bits << (uint32_t)(e0 & 31)) : 0u;
#pragma unroll
    for (int o = 1; o < LPW; o <<= 1) w |= (uint32_t)__shfl_xor((int)w, o, 64);
    // the tile's mask words were zeroed at entry: only words with set bits are written
    if (w != 0u && ((tid & 63) % LPW) == 0) {
      const int64_t wi = e0 >> 5;
      const bool whole = (wi * 32 >= g.sstart) && (wi * 32 + 32 <= g.te);
      if (whole) d.free_mask[wi] = w;
      else atomicOr(&d.free_mask[wi], w);
    }
  };

  for (;;) {
    if (sh.phase == PH_DONE) break;
    const int ph = sh.phase;
    double* pb = d.part + (size_t)buf * VMAX * TILES_PAD;
    const uint64_t t_pass0 = clk();
    trace_put(d, pass_no, 0, ((uint64_t)ph << 56) | (t_pass0 & 0x00ffffffffffffffull));
    int nv = 0;
    uint64_t maxmask = 0;
    // compacted tiles of this workgroup (every wave kept its pairs): they are
    // evaluated one per wave after the loop below
    const int nloc = wid < d.ntiles ? (d.ntiles - wid + G - 1) / G : 0;
    if (ph == PH_SEARCH && CB != nullptr) {
      for (int k = tid; k < nloc; k += BLOCK) {
        const int tile = wid + k * G;
        const TileGeom g = tile_geom<T>(d, tile);
        bool f = g.interior && sh.S.cmode[g.seg] == 2 && sh.S.state[g.seg] == SEG_SEARCH;
        if (f) {
          double c[NWAVE];
#pragma unroll
          for (int w = 0; w < NWAVE; ++w) c[w] = fetch_published(meta_row(d, w) + tile);
#pragma unroll
          for (int w = 0; w < NWAVE; ++w) f = f && c[w] >= 0.0;
        }
        sh.cflag[k] = f ? 1 : 0;
      }
      __syncthreads();
    }

    for (int tile = wid; tile < d.ntiles; tile += G) {
      const TileGeom g = tile_geom<T>(d, tile);
      const int s = g.seg;
      if (ph == PH_ZERO) {
        // rows held at equality (Sec. 3.2) also need the bracket of the
        // opposite direction: the EQ instantiation adds its two sums
        auto zero_tile = [&]() __attribute__((always_inline)) {
          constexpr int NZ = EQ ? 9 : 7;
          constexpr int ZA = NZ - 1;         // max |a|
          nv = NZ;
          maxmask = (EQ ? ((1ull << 2) | (1ull << 6)) : (1ull << 2)) | (1ull << ZA);
          // lam = 0: a.clip(y), slope, largest breakpoint, saturated sum, sum |a|,
          // non-finite count [, largest opposite breakpoint, sum a . other bound], max |a|
          double acc[NZ];
#pragma unroll
          for (int v = 0; v < NZ; ++v) acc[v] = (v == 2 || (EQ && v == 6)) ? -INFINITY : 0.0;
          // lam = 0: a.clip(y), slope, largest breakpoint, saturated sum, sum |a|, non-finite count
          auto zero_elem = [&](double y, double av) __attribute__((always_inline)) {
            const double x0 = clampd(y, lo, hi);
            acc[0] = fma(av, x0, acc[0]);
            if (y >= lo && y <= hi) acc[1] = fma(av, av, acc[1]);
            if (av != 0.0) {
              const double bound = (av > 0.0) ? lo : hi;
              const double r = recip(av);
              acc[2] = fmax(acc[2], (y - bound) * r);
              acc[3] = fma(av, bound, acc[3]);
              if constexpr (EQ) {
                // the opposite direction (lam < 0) of an equality row: the
                // element moves to the other bound
                const double other = (av > 0.0) ? hi : lo;
                acc[6] = fmax(acc[6], (other - y) * r);
                acc[7] = fma(av, other, acc[7]);
              }
            }
            acc[4] += fabs(av);
            acc[ZA] = fmax(acc[ZA], fabs(av));
            if (!isfinite(y) || !isfinite(av)) acc[5] += 1.0;
          };
          if (tile == wid && g.nsweep <= RS) {
            // load (pgd: form) this workgroup's first tile into registers
            const double beta = sh.pg.beta, step = d.omega * sh.pg.alpha;
            {
              int64_t re0[RS];
  #pragma unroll
              for (int k = 0; k < RS; ++k) {
                bool full; uint32_t mask;
                rslot(g, k, re0[k], full, mask);
                if (!mask) re0[k] = d.n;        // reads zeros
              }
              if (d.pgd) {
                T tmp[RS][1][V];
                const T* pa[1] = {A};
                ld_slots<T, RS, 1, NT>(pa, re0, d.n, tmp);
  #pragma unroll
                for (int k = 0; k < RS; ++k)
  #pragma unroll
                  for (int q = 0; q < V; ++q) ra[k][q] = tmp[k][0][q];
              } else {
                T tmp[RS][2][V];
                const T* pa[2] = {A, Y};
                ld_slots<T, RS, 2, NT>(pa, re0, d.n, tmp);
  #pragma unroll
                for (int k = 0; k < RS; ++k)
  #pragma unroll
                  for (int q = 0; q < V; ++q) { ra[k][q] = tmp[k][0][q]; ry[k][q] = tmp[k][1][q]; }
              }
            }
            if (d.pgd) {
              // Alg. 3: d_t = -grad f + beta d_{t-1}; rho~ = rho_t + omega alpha_t d_t
              // in the stream precision; rho~ stays in registers.
              // the loads of slot k + 1 are issued before d_t of slot k is
              // stored (the store may alias them)
              T nr[V], ng[V], nd[V];
              auto fetch = [&](int k) __attribute__((always_inline)) {
                int64_t e0 = d.n;               // reads zeros
                if (k < RS) {
                  bool full; uint32_t mask;
                  rslot(g, k, e0, full, mask);
                  if (!mask) e0 = d.n;
                }
                T tmp[1][3][V];
                const T* pa[3] = {(const T*)d.rho, (const T*)d.grad, d.zero_step ? (const T*)d.rho : (const T*)d.dir};
                ld_slots<T, 1, 3, NT>(pa, &e0, d.n, tmp);
  #pragma unroll
                for (int q = 0; q < V; ++q) {
                  nr[q] = tmp[0][0][q];
                  ng[q] = tmp[0][1][q];
                  nd[q] = d.zero_step ? (T)0 : tmp[0][2][q];
                }
              };
              fetch(0);
  #pragma unroll
              for (int k = 0; k < RS; ++k) {
                T rr[V], rg[V], rd[V], dn[V];
  #pragma unroll
                for (int q = 0; q < V; ++q) { rr[q] = nr[q]; rg[q] = ng[q]; rd[q] = nd[q]; }
                fetch(k + 1);
                int64_t e0; bool full; uint32_t mask;
                rslot(g, k, e0, full, mask);
                if (!mask) continue;
  #pragma unroll
                for (int q = 0; q < V; ++q) {
                  const double dd = d.zero_step ? -f64(rg[q]) : fma(beta, f64(rd[q]), -f64(rg[q]));
                  dn[q] = (T)dd;
                  ry[k][q] = (T)fma(step, dd, f64(rr[q]));
                }
                st_vec<T>((T*)d.dir, e0, mask, full, dn);
              }
            }
            rbits = 0u;
  #pragma unroll
            for (int k = 0; k < RS; ++k) {
              int64_t e0; bool full; uint32_t mask;
              rslot(g, k, e0, full, mask);
              rbits |= mask << (k * V);
  #pragma unroll
              for (int q = 0; q < V; ++q) {
                // elements outside the segment contribute exactly zero from here on
                if (!(mask & (1u << q))) { ra[k][q] = (T)0; ry[k][q] = (T)0; }
                else zero_elem(f64(ry[k][q]), f64(ra[k][q]));
              }
            }
            resident = true;
          } else if (d.pgd) {
            // Alg. 3: d_t = -grad f + beta d_{t-1}; rho~ = rho_t + omega alpha_t d_t,
            // materialized in the stream precision (it is the point projected).
            T* Dw = (T*)d.dir;
            const double beta = sh.pg.beta, step = d.omega * sh.pg.alpha;
            auto body = [&](const T* a, const T* r, const T* gr, const T* dp, int64_t e0, uint32_t mask, bool full)
                __attribute__((always_inline)) {
              T dn[V], rt[V];
  #pragma unroll
              for (int q = 0; q < V; ++q) {
                const double dd = dp ? fma(beta, f64(dp[q]), -f64(gr[q])) : -f64(gr[q]);
                dn[q] = (T)dd;
                rt[q] = (T)fma(step, dd, f64(r[q]));
              }
              st_vec<T>(Dw, e0, mask, full, dn);
              st_vec<T>(X, e0, mask, full, rt);
  #pragma unroll
              for (int q = 0; q < V; ++q)
                if (mask & (1u << q)) zero_elem(f64(rt[q]), f64(a[q]));
            };
            if (d.zero_step) {
              const T* ptr[3] = {A, (const T*)d.rho, (const T*)d.grad};
              stream_tile<T, 3, SU1, NT>(g, d.n, ptr, [&](const T (&b)[3][V], int64_t e0, uint32_t mask, bool full) __attribute__((always_inline)) {
                body(b[0], b[1], b[2], nullptr, e0, mask, full);
              });
            } else {
              const T* ptr[4] = {A, (const T*)d.rho, (const T*)d.grad, (const T*)d.dir};
              stream_tile<T, 4, SU1, NT>(g, d.n, ptr, [&](const T (&b)[4][V], int64_t e0, uint32_t mask, bool full) __attribute__((always_inline)) {
                body(b[0], b[1], b[2], b[3], e0, mask, full);
              });
            }
          } else {
            const T* ptr[2] = {Y, A};
            stream_tile<T, 2, SU, NT>(g, d.n, ptr, [&](const T (&b)[2][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
  #pragma unroll
              for (int q = 0; q < V; ++q)
                if (mask & (1u << q)) zero_elem(f64(b[0][q]), f64(b[1][q]));
            });
          }
          block_to_part<NZ>(acc, nv, maxmask, sh.red, pb, tile);
        };
        zero_tile();
      } else if (ph == PH_SEARCH) {
        nv = NV_SEARCH; maxmask = 0;
        if (sh.S.state[s] == SEG_DONE) continue;      // finished segments are not streamed
        const double sgs = EQ ? sh.sg[s] : 1.0;
        const double l0 = sgs * sh.S.trial[s][0], l1 = sgs * sh.S.trial[s][1];
        // phi(lam_t) + b = a.clip(y - lam_t a) and its slope sum_free a^2, per trial;
        // elements outside the segment enter with a = 0, y = 0 and add nothing.
        // Two chains per sum (even and odd element of a vector), added at the
        // end of the tile.  The slope only steers the choice of trial points,
        // so with float streams it is summed in float (a^2 exact in float
        // up to rounding; a thread adds at most 32 terms per tile).
        using S = typename std::conditional<sizeof(T) == 4, float, double>::type;
        double cs[2][2] = {{0, 0}, {0, 0}};     // [chain][trial]
        S sl[2][2] = {{0, 0}, {0, 0}};
        auto run = [&](auto two_c) __attribute__((always_inline)) {
          constexpr bool TWO = decltype(two_c)::value;
          auto elem = [&](T yt, T at, int c) __attribute__((always_inline)) {
            const double yq = f64(yt), av = f64(at);
            const S a2 = (S)at * (S)at;
            const double z0 = fma(-l0, av, yq);
            const double x0 = fmin(fmax(z0, lo), hi);
            cs[c][0] = fma(av, x0, cs[c][0]);
            sl[c][0] += (x0 == z0) ? a2 : (S)0;     // free: the clip left z unchanged
            if constexpr (TWO) {
              const double z1 = fma(-l1, av, yq);
              const double x1 = fmin(fmax(z1, lo), hi);
              cs[c][1] = fma(av, x1, cs[c][1]);
              sl[c][1] += (x1 == z1) ? a2 : (S)0;
            }
          };
          if (tile == wid && resident) {
#pragma unroll
            for (int k = 0; k < RS; ++k)
#pragma unroll
              for (int q = 0; q < V; ++q) elem(ry[k][q], ra[k][q], q & 1);
          } else {
            const T* ptr[2] = {Y, A};
            stream_tile<T, 2, SU, NT>(g, d.n, ptr, [&](const T (&b)[2][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
              for (int q = 0; q < V; ++q) {
                const bool ok = (mask >> q) & 1u;
                elem(ok ? b[0][q] : (T)0, ok ? b[1][q] : (T)0, q & 1);
              }
            });
          }
        };
        double kept = 0.0;                        // pairs this thread's wave kept (compaction pass)
        const int cm = (CB != nullptr && g.interior) ? sh.S.cmode[s] : 0;
        if (cm == 2 && sh.cflag[(tile - wid) / G]) continue;     // evaluated by one wave below
        if (cm == 1) {
          // this pass evaluates the trials as usual and compacts the tile
          // against the bracket it starts from (every later trial lies in it);
          // wave w owns elements of threads [64 w, 64 w + 64) and the region
          // [w E / NWAVE, (w + 1) E / NWAVE) of the tile's scratch, E = tile_elems
          const double ba = sgs * sh.S.lo[s], bb = sgs * sh.S.hi[s];
          const double bl = fmin(ba, bb), bh = fmax(ba, bb);
          const int64_t seg_el = d.tile_elems / NWAVE;
          T* dst = CB + g.ts + (int64_t)(tid >> 6) * seg_el;
          int64_t crun = 0;
          bool cok = true;
          double s0 = 0.0, qq = 0.0;
          auto slot_c = [&](const T* yv, const T* av, auto two_c) __attribute__((always_inline)) {
            constexpr bool TWO = decltype(two_c)::value;
            uint32_t ub = 0u;
#pragma unroll
            for (int q = 0; q < V; ++q) {
              const double yq = f64(yv[q]), aq = f64(av[q]);
              const S a2 = (S)av[q] * (S)av[q];
              const double z0 = fma(-l0, aq, yq);
              const double x0 = fmin(fmax(z0, lo), hi);
              cs[q & 1][0] = fma(aq, x0, cs[q & 1][0]);
              sl[q & 1][0] += (x0 == z0) ? a2 : (S)0;
              if constexpr (TWO) {
                const double z1 = fma(-l1, aq, yq);
                const double x1 = fmin(fmax(z1, lo), hi);
                cs[q & 1][1] = fma(aq, x1, cs[q & 1][1]);
                sl[q & 1][1] += (x1 == z1) ? a2 : (S)0;
              }
              // branch-free: decided elements fold into s0 (and qq when free)
              const int sa = elem_state(yq, aq, bl, lo, hi), sb = elem_state(yq, aq, bh, lo, hi);
              const bool dec = sa == sb, fr = dec && sa == 1;
              const double term = fr ? yq : (sa == 0 ? lo : hi);
              s0 = dec ? fma(aq, term, s0) : s0;
              qq = fr ? fma(aq, aq, qq) : qq;
              ub |= dec ? 0u : (1u << q);
            }
            compact_slot<T>(yv, av, ub, dst, seg_el / 2, crun, cok);
          };
          auto run_k = [&](auto two_c) __attribute__((always_inline)) {
            if (tile == wid && resident) {
#pragma unroll 1
              for (int k = 0; k < RS; ++k) slot_c(ry[k], ra[k], two_c);
            } else {
              // an interior tile: every slot whole (nsweep even), two slots in flight
              const int64_t base = (g.p0 + (int64_t)tid) * V;
              for (int k0 = 0; k0 < g.nsweep; k0 += 2) {
                T b[2][2][V];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                  const int64_t e0 = base + (int64_t)(k0 + u) * (BLOCK * V);
                  ld_vec_whole<T, NT>(gptr(Y), e0, b[u][0]);
                  ld_vec_whole<T, NT>(gptr(A), e0, b[u][1]);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) slot_c(b[u][0], b[u][1], two_c);
              }
            }
          };
          if (l1 == l1) run_k(std::true_type{}); else run_k(std::false_type{});
          // the wave's folded sums and count (fixed butterfly order)
          s0 = wave_sum(s0);
          qq = wave_sum(qq);
          if ((tid & 63) == 0) {
            const int w = tid >> 6;
            publish(meta_row(d, w) + tile, cok ? (double)crun : -1.0);
            publish(meta_row(d, NWAVE + w) + tile, s0);
            publish(meta_row(d, 2 * NWAVE + w) + tile, qq);
            kept = cok ? (double)crun : 0.0;
          }
        } else {
          if (l1 == l1) run(std::true_type{}); else run(std::false_type{});
        }
        const double acc[NV_SEARCH] = {cs[0][0] + cs[1][0], (double)sl[0][0] + (double)sl[1][0],
                                       cs[0][1] + cs[1][1], (double)sl[0][1] + (double)sl[1][1], kept};
        block_to_part<NV_SEARCH>(acc, nv, maxmask, sh.red, pb, tile);
      } else {  // PH_FINAL
        nv = NV_FINAL1; maxmask = 0;
        double acc[NV_FINAL1] = {0, 0, 0, 0, 0};
        const double lam = (EQ ? sh.sg[s] : 1.0) * sh.S.lam[s];
        const T* R = (const T*)d.rho;
        // x = clip(y - lam a) in the stream precision; a.x, free count, pgd norms
        auto final_slot = [&](const T* yv, const T* a, const T* r, int64_t e0, uint32_t mask, bool full) __attribute__((always_inline)) -> uint32_t {
          uint32_t bits = 0;
          T xo[V];
#pragma unroll
          for (int q = 0; q < V; ++q) {
            const double z = fma(-lam, f64(a[q]), f64(yv[q]));
            xo[q] = (T)clampd(z, lo, hi);
            if (!(mask & (1u << q))) continue;
            const double xr = (double)xo[q];
            acc[0] = fma(f64(a[q]), xr, acc[0]);
            if (z >= lo && z <= hi) { acc[1] += 1.0; bits |= 1u << q; }
            if (d.pgd) {
              const double df = xr - f64(r[q]);
              acc[2] = fma(df, df, acc[2]);
              acc[3] = fma(xr, xr, acc[3]);
            }
            const double dy = xr - f64(yv[q]);            // distance of the projection
            acc[4] = fma(dy, dy, acc[4]);
          }
          st_vec<T>(X, e0, mask, full, xo);
          return bits;
        };
        if (tile == wid && resident) {
          // rho_t of slot k + 1 is requested before x of slot k is stored
          // (the store may alias it), so the loads overlap the slot work
          T rnext[V];
          auto fetch_r = [&](int k) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < V; ++q) rnext[q] = (T)0;
            if (d.pgd && k < RS) {
              int64_t e0;
              bool full; uint32_t mask;
              rslot(g, k, e0, full, mask);
              if (!rmask(k)) e0 = d.n;          // reads zeros
              T tmp[1][1][V];
              const T* pa[1] = {R};
              ld_slots<T, 1, 1, NT>(pa, &e0, d.n, tmp);
#pragma unroll
              for (int q = 0; q < V; ++q) rnext[q] = tmp[0][0][q];
            }
          };
          fetch_r(0);
#pragma unroll
          for (int k = 0; k < RS; ++k) {
            T rcur[V];
#pragma unroll
            for (int q = 0; q < V; ++q) rcur[q] = rnext[q];
            fetch_r(k + 1);
            int64_t e0; bool full; uint32_t mask;
            rslot(g, k, e0, full, mask);
            mask = rmask(k);
            const bool any = mask != 0u;
            const uint32_t bits = any ? final_slot(ry[k], ra[k], rcur, e0, mask, full) : 0u;
            if (d.free_mask) put_mask(any, e0, bits, g);
          }
        } else {
          // one slot ahead: the loads of slot k + 1 are issued before the
          // store of slot k (x may alias y)
          T ny[V], na[V], nr[V];
          int64_t ne0 = 0; bool nfull = false, nany = false; uint32_t nmask = 0u;
          auto fetch = [&](int k) __attribute__((always_inline)) {
            // a slot with no element of this segment keeps its own position:
            // put_mask addresses the word of 8 lanes by the first lane's
            // position, and at a block start that lane may hold only
            // elements of the previous block
            ne0 = 0;
            nany = (k < g.nsweep) && slot<T>(g, k, ne0, nfull, nmask);
            if (!nany) { nmask = 0u; nfull = false; }
            int64_t le0 = nany ? ne0 : d.n;    // reads zeros
            T tmp[1][3][V];
            const T* pa[3] = {Y, A, d.pgd ? R : Y};
            ld_slots<T, 1, 3, NT>(pa, &le0, d.n, tmp);
#pragma unroll
            for (int q = 0; q < V; ++q) {
              ny[q] = tmp[0][0][q];
              na[q] = tmp[0][1][q];
              nr[q] = d.pgd ? tmp[0][2][q] : (T)0;
            }
          };
          fetch(0);
          for (int k = 0; k < g.nsweep; ++k) {
            T yv[V], a[V], r[V];
#pragma unroll
            for (int q = 0; q < V; ++q) { yv[q] = ny[q]; a[q] = na[q]; r[q] = nr[q]; }
            const int64_t e0 = ne0; const bool full = nfull, any = nany; const uint32_t mask = nmask;
            fetch(k + 1);
            const uint32_t bits = any ? final_slot(yv, a, r, e0, mask, full) : 0u;
            if (d.free_mask) put_mask(any, e0, bits, g);
          }
        }
        block_to_part<NV_FINAL1>(acc, nv, maxmask, sh.red, pb, tile);
      }
    }
    if (ph == PH_SEARCH && CB != nullptr) {
      // one wave per compacted tile: its folded sums plus the kept pairs, the
      // pairs of the tile's NWAVE regions taken in order, 8 per lane in flight
      using S = typename std::conditional<sizeof(T) == 4, float, double>::type;
      const int w = tid >> 6, lane = tid & 63;
      const int64_t seg_el = d.tile_elems / NWAVE;
      int rank = 0;
      for (int k = 0; k < nloc; ++k) {
        if (!sh.cflag[k]) continue;
        if ((rank++ % NWAVE) != w) continue;
        const int tile = wid + k * G;
        const TileGeom g = tile_geom<T>(d, tile);
        const int s = g.seg;
        const double sgs = EQ ? sh.sg[s] : 1.0;
        const double l0 = sgs * sh.S.trial[s][0], l1 = sgs * sh.S.trial[s][1];
        const bool two = (l1 == l1);
        const double mv = lane < META_ROWS ? fetch_published(meta_row(d, lane) + tile) : 0.0;
        int64_t pre[NWAVE + 1];
        pre[0] = 0;
        double S0 = 0.0, Q = 0.0;
#pragma unroll
        for (int v = 0; v < NWAVE; ++v) pre[v + 1] = pre[v] + (int64_t)__shfl(mv, v, 64);
#pragma unroll
        for (int v = 0; v < NWAVE; ++v) S0 += __shfl(mv, NWAVE + v, 64);
#pragma unroll
        for (int v = 0; v < NWAVE; ++v) Q += __shfl(mv, 2 * NWAVE + v, 64);
        const T* base = CB + g.ts;
        double c0 = 0.0, c1 = 0.0;
        S f0 = 0, f1 = 0;
        constexpr int PB = 8;
        for (int64_t j0 = 0; j0 < pre[NWAVE]; j0 += 64 * PB) {
          T yy[PB], aa[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int64_t j = j0 + (int64_t)u * 64 + lane;
            yy[u] = (T)0;
            aa[u] = (T)0;
            // the region holding pair j (constant indices keep pre in registers)
            int v = 0;
            int64_t pv = 0;
#pragma unroll
            for (int r = 1; r < NWAVE; ++r) {
              const bool ge = j >= pre[r];
              v += ge ? 1 : 0;
              pv = ge ? pre[r] : pv;
            }
            if (j < pre[NWAVE]) get_pair<T>(base + (int64_t)v * seg_el, j - pv, yy[u], aa[u]);
          }
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const double yq = f64(yy[u]), av = f64(aa[u]);
            const S a2 = (S)aa[u] * (S)aa[u];
            const double z0 = fma(-l0, av, yq);
            const double x0 = fmin(fmax(z0, lo), hi);
            c0 = fma(av, x0, c0);
            f0 += (x0 == z0) ? a2 : (S)0;
            if (two) {
              const double z1 = fma(-l1, av, yq);
              const double x1 = fmin(fmax(z1, lo), hi);
              c1 = fma(av, x1, c1);
              f1 += (x1 == z1) ? a2 : (S)0;
            }
          }
        }
        // padding pairs (0, 0) add exactly nothing: z = 0 is clipped (x = lo
        // or 0 times a = 0) and the slope term is a^2 = 0
        c0 = wave_sum(c0);
        c1 = wave_sum(c1);
        const double g0 = wave_sum((double)f0), g1 = wave_sum((double)f1);
        if (lane == 0) {
          publish(&pb[0 * TILES_PAD + tile], c0 + fma(-l0, Q, S0));
          publish(&pb[1 * TILES_PAD + tile], g0 + Q);
          publish(&pb[2 * TILES_PAD + tile], two ? c1 + fma(-l1, Q, S0) : 0.0);
          publish(&pb[3 * TILES_PAD + tile], two ? g1 + Q : 0.0);
          publish(&pb[4 * TILES_PAD + tile], 0.0);
        }
      }
      wait_own_stores();
    }
    if (ph == PH_ZERO) { nv = EQ ? 9 : 7; maxmask = (EQ ? ((1ull << 2) | (1ull << 6)) : (1ull << 2)) | (1ull << (nv - 1)); }
    else if (ph == PH_SEARCH) { nv = NV_SEARCH; maxmask = 0; }
    else { nv = NV_FINAL1; maxmask = 0; }

    trace_put(d, pass_no, 1, clk());
    trace_wg(d, pass_no, t_pass0, clk());
    if (!grid_reduce(d, d.epoch0 + (uint64_t)pass_no + 1, pb, nv, maxmask, d.nseg, sh.tot, &sh.abort_flag, pass_no)) break;
    trace_put(d, pass_no, 4, clk());

    // ---------------- control (identical in every workgroup)
    if (ph == PH_ZERO) {
      constexpr int zs = EQ ? 9 : 7;
      if (d.auto_tau > 0.0) kappa = auto_kappa(d.auto_tau, &sh.tot[2], zs, d.nseg);
      for (int s = tid; s < d.nseg; s += BLOCK) {
        const double* t = &sh.tot[s * zs];
        sh.amax[s] = t[zs - 1];
        double scale = t[4] * fmax(fabs(lo), fabs(hi));
        if (!(scale > 0.0)) scale = 1.0;
        const bool eq = EQ && ((d.eq_mask >> s) & 1ull);
        const double f0 = t[0] - sh.bs[s];
        if (t[5] > 0.0) {
          sh.S.lam[s] = 0.0; sh.S.outcome[s] = PGDTO_NONFINITE; sh.S.state[s] = SEG_DONE;
          sh.S.npass[s] = 0; sh.S.width[s] = 0.0; sh.S.scale[s] = scale;
          sh.S.err[s] = NAN; sh.S.slope[s] = 0.0;
        } else if (eq && f0 < 0.0) {
          // equality row below its target (Sec. 3.2): the opposite
          // inequality (-a).x <= -b is the active one; search it for
          // lam' >= 0 and report lam = -lam'
          sh.sg[s] = -1.0;
          if constexpr (EQ) {
            if (search_init(sh.S, s, -f0, t[1] + kappa, t[6], -t[7], -sh.bs[s], kappa, scale, d.search, true) &&
                d.warm)
              search_warm(sh.S, s, -d.lam0[s]);
          }
        } else {
          if (search_init(sh.S, s, f0, t[1] + kappa, t[2], t[3], sh.bs[s], kappa, scale, d.search, true) && d.warm)
            search_warm(sh.S, s, d.lam0[s]);
          if (eq && sh.S.outcome[s] == PGDTO_INACTIVE) sh.S.outcome[s] = PGDTO_CONVERGED;   // h(0) = 0
        }
      }
      __syncthreads();
      if (tid == 0) {
        sh.passes += 1;
        int any = 0;
        for (int s = 0; s < d.nseg; ++s) any |= (sh.S.state[s] == SEG_SEARCH);
        sh.phase = any ? PH_SEARCH : PH_FINAL;
      }
    } else if (ph == PH_SEARCH) {
      for (int s = tid; s < d.nseg; s += BLOCK) {
        if (sh.S.state[s] != SEG_SEARCH) continue;
        const double sg = EQ ? sh.sg[s] : 1.0;      // a sign-flipped row sees -a.x and -b
        const double* t = &sh.tot[s * NV_SEARCH];
        if (sh.S.cmode[s] == 2) sh.npc[s] += 1;
        search_update(sh.S, s, sg * t[0], sg * t[2], t[1], t[3], sg * sh.bs[s], kappa, d.tol_n, d.tol_b,
                      d.max_search, d.search, true);
        // free-set compaction: done in the pass just finished, or due in the
        // next one once the bracket lies within 25% of its upper end
        if (sh.S.cmode[s] == 1) { sh.S.cmode[s] = 2; sh.ncomp[s] = t[4]; }
        else if (sh.S.cmode[s] == 0 && d.compact && d.cbuf && sh.S.state[s] == SEG_SEARCH &&
                 sh.S.hi[s] - sh.S.lo[s] <= 0.25 * fabs(sh.S.hi[s]))
          sh.S.cmode[s] = 1;
      }
      __syncthreads();
      if (tid == 0) {
        sh.passes += 1;
        int any = 0;
        for (int s = 0; s < d.nseg; ++s) any |= (sh.S.state[s] == SEG_SEARCH);
        sh.phase = any ? PH_SEARCH : PH_FINAL;
      }
    } else {  // PH_FINAL: results (workgroup 0 writes)
      if (wid == 0) {
        pgdto_result* R = d.pgd ? &((pgdto_pgd_out*)d.result)->proj : (pgdto_result*)d.result;
        for (int s = tid; s < d.nseg; s += BLOCK) {
          const double lam_s = (EQ ? sh.sg[s] : 1.0) * sh.S.lam[s];
          const double r = sh.tot[s * NV_FINAL1 + 0] - sh.bs[s];
          R->lambda[s] = lam_s;
          R->resid[s] = r;
          R->slack[s] = kappa * lam_s;
          R->row_outcome[s] = sh.S.outcome[s];
          const double le = lam_error(lam_s, sh.S.err[s], sh.S.scale[s], sh.S.slope[s]);
          R->lambda_err[s] = le;
          sh.red[PGDTO_MAX_BLOCKS + s] = le;
          // scaled KKT residual of the stored x (equality rows: always active)
          const double h = r - kappa * lam_s;
          const bool act = (lam_s != 0.0) || (EQ && ((d.eq_mask >> s) & 1ull));
          sh.red[s] = (act ? fabs(h) : fmax(h, 0.0)) / sh.S.scale[s];
        }
        __syncthreads();
        if (tid == 0) {
          int worst = PGDTO_INACTIVE, anyact = 0, np = 0;
          double nfree = 0.0, diff2 = 0.0, xx = 0.0, wmax = 0.0, rmax = 0.0, xerr = 0.0, ncomp = -1.0, dist2 = 0.0;
          int npc = 0;
          for (int s = 0; s < d.nseg; ++s) {
            if (severity(sh.S.outcome[s]) > severity(worst)) worst = sh.S.outcome[s];
            anyact |= (sh.S.outcome[s] != PGDTO_INACTIVE);
            np = max(np, sh.S.npass[s]);
            wmax = fmax(wmax, sh.S.width[s]);
            rmax = fmax(rmax, sh.red[s]);
            // blocks are disjoint: the element error is the largest block's
            xerr = fmax(xerr, sh.amax[s] * sh.red[PGDTO_MAX_BLOCKS + s]);
            nfree += sh.tot[s * NV_FINAL1 + 1];
            diff2 += sh.tot[s * NV_FINAL1 + 2];
            xx += sh.tot[s * NV_FINAL1 + 3];
            dist2 += sh.tot[s * NV_FINAL1 + 4];
            if (sh.ncomp[s] >= 0.0) ncomp = fmax(ncomp, 0.0) + sh.ncomp[s];
            npc = max(npc, sh.npc[s]);
          }
          R->n_compact = (int64_t)ncomp;
          R->passes_compacted = npc;
          R->dist2 = dist2;
          R->outcome = worst;
          R->error = 0;
          R->path = anyact ? 1 : 0;
          R->passes = sh.passes + 1;
          R->iters_search = np;
          R->iters_newton = 0;
          R->iters_ls = 0;
          R->m = d.nseg;
          R->n_free = (int64_t)nfree;
          R->res_inf = rmax;
          R->lambda_width = wmax;
          R->kappa = kappa;
          R->x_err = xerr + half_ulp(fmax(fabs(lo), fabs(hi)), sizeof(T) == 4);
          if (d.pgd) {
            pgdto_pgd_out* P = (pgdto_pgd_out*)d.result;
            P->alpha = sh.pg.alpha;
            P->beta = sh.pg.beta;
            P->used_fallback = sh.pg.used_fb;
            P->rel_change = (xx > 0.0) ? sqrt(diff2) / sqrt(xx) : INFINITY;
            P->converged = (P->rel_change <= d.tol_stop) ? 1 : 0;
          }
        }
      }
      if (tid == 0) sh.phase = PH_DONE;
    }
    __syncthreads();
    trace_put(d, pass_no, 5, clk());
    ++pass_no;
    buf ^= 1;
    if (sh.phase == PH_DONE) break;
  }
  int32_t* errp = nullptr;
  if (d.result) errp = d.pgd ? &((pgdto_pgd_out*)d.result)->proj.error : &((pgdto_result*)d.result)->error;
  report_error(d, errp);
  if (buf_end && threadIdx.x == 0) *buf_end = buf;     // the next instance of a batch slot starts there
}

// Zero the free-mask words of this workgroup's tiles (before the first grid
// barrier; the final pass sets bits only where elements are free).  A word at
// a block boundary belongs to two tiles, whose workgroups may sit on
// different XCDs and both set bits in it with device atomics: the zeros are
// written through to memory and complete before the first barrier, so that
// no dirty zero is left in an L2 to be written back over those bits.
template <typename T>
__device__ __forceinline__ void clear_mask_tiles(const Desc& d) {
  if (!d.free_mask) return;
  const int wid = wg_id(d), G = wg_num(d);
  for (int tile = wid; tile < d.ntiles; tile += G) {
    const TileGeom g = tile_geom<T>(d, tile);
    const int64_t w0 = g.ts >> 5, w1 = (g.te + 31) >> 5;
    for (int64_t w = w0 + threadIdx.x; w < w1; w += BLOCK)
      __hip_atomic_store(&d.free_mask[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  wait_own_stores();
}

template <typename T, bool EQ, bool CP>
__global__ __launch_bounds__(BLOCK, 2) void k_solve_1d(const Desc) {
  __shared__ Sh1D sh;
  __shared__ Desc sd;
  __shared__ int32_t late;
  load_desc(sd);
  if (!enter_launch(sd, &late)) return;
  clear_mask_tiles<T>(sd);
  solve_1d<T, EQ, CP>(sh, sd);
}

// ================================================================== coupled kernel
// Algorithm 2: Stage 1 (m lockstep single-row searches of the regularized
// 1-row problem, then one pass checking every candidate lam_j* e_j against
// all rows), Stage 2 (semismooth Newton on the m duals with the Jacobian
// A D A^T + kappa I of eq. reg_jacobian and a line search on M = |Phi|^2/2).

template <int M> struct CN {
  static constexpr int NJ = M * (M + 1) / 2;
  static constexpr bool FUSE = (M <= 3);
  static constexpr int NV_R = 7 + M;
  static constexpr int NV_ZERO = 6 * M + 1;      // ..., non-finite count, then max |a_j| per row
  static constexpr int NV_S1 = 2 * NT * M;
  static constexpr int NV_NEWTON = M + NJ;
  static constexpr int NV_CHECK = M * M + (FUSE ? NV_NEWTON : 0);
  static constexpr int NV_FINAL = M + 4;         // a.x per row, free count, pgd norms, |x - y|^2
  static constexpr int U = (M <= 2) ? 4 : 2;     // vector slots in flight per chunk
  static constexpr int NVM = NV_CHECK > NV_ZERO ? (NV_CHECK > NV_S1 ? NV_CHECK : NV_S1) : (NV_ZERO > NV_S1 ? NV_ZERO : NV_S1);
};

struct NewtonState {
  double lam[SMALL_M], h[SMALL_M], J[SMALL_M * SMALL_M];   // current iterate
  double delta[SMALL_M], phi2, M0;                                    // direction, |Phi|^2, merit
  double trial[SMALL_M], gamma;
  double blam[SMALL_M], bh[SMALL_M], bJ[SMALL_M * SMALL_M];  // best Armijo trial
  int32_t have_best, ls, it, init;   // init: next Newton pass is the starting evaluation
  double lam1[SMALL_M];          // Stage-1 candidates
  double h0[SMALL_M];
};

struct ShC {
  double tot[VMAX];
  double red[NWAVE * BLOCK];
  double bs[SMALL_M];
  Search S;
  NewtonState N;
  PgdScalars pg;
  CtlParams P;
  double lamf[SMALL_M];    // multiplier used by the final pass
  double lerr[SMALL_M];    // stated |lam - lam*| estimate at exit (before the rounding allowance)
  double lslope[SMALL_M];  // diagonal of (A D A^T + kappa I) or the 1-D slope at exit
  double amax[SMALL_M];    // max_i |a_ji| (zero pass)
  double asum[SMALL_M];    // sum_i |a_ji| (zero pass)
  double res_inf;
  int32_t phase, abort_flag, passes, path, outcome, nonfinite, s1passes, pad;
};

// Unpack the symmetric Jacobian sums (upper triangle, row-major) into J[j][k].
template <int M>
__device__ __forceinline__ void unpack_J(const double* src, double* J) {
  int q = 0;
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int k = j; k < M; ++k) { J[j * SMALL_M + k] = src[q]; J[k * SMALL_M + j] = src[q]; ++q; }
}

// Continuous NCP: Phi_j = max(h_j, -c_j lam_j), c_j = J_jj + kappa, active if
// h_j + c_j lam_j > 0.  Paper NCP (eq. phi): active if h_j > 0, Phi_j = h_j;
// else Phi_j = -lam_j if h_j < 0, 0 if h_j = 0.  Equality rows (Sec. 3.2):
// always active, Phi_j = h_j.
template <int M>
__device__ __forceinline__ void ncp(const double* h, const double* J, const double* lam, double kappa,
                                    int mode, int eq, double* phi, bool* act) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if ((eq >> j) & 1) {
      act[j] = true;
      phi[j] = h[j];
    } else if (mode == PGDTO_NCP_PAPER) {
      act[j] = h[j] > 0.0;
      phi[j] = act[j] ? h[j] : (h[j] < 0.0 ? -lam[j] : 0.0);
    } else {
      const double c = J[j * SMALL_M + j] + kappa;
      act[j] = h[j] + c * lam[j] > 0.0;
      phi[j] = act[j] ? h[j] : -c * lam[j];
    }
  }
}

// Solve the semismooth Newton system J_Phi Delta = Phi (Appendix A.2): rows
// outside the active set release their multiplier (Delta_j = -lam_j, or 0 on
// the paper NCP's h_j = 0 branch); active rows solve
// (J + kappa I)_SS Delta_S = h_S - (J + kappa I)_SN Delta_N by Cholesky.
template <int M>
__device__ __forceinline__ void newton_direction(const double* h, const double* J, const double* lam, double kappa,
                                 const bool* act, const double* phi, int mode, double* delta) {
  double K[M][M], r[M], inv[M];
#pragma unroll
  for (int j = 0; j < M; ++j) delta[j] = act[j] ? 0.0 : (mode == PGDTO_NCP_PAPER ? phi[j] : -lam[j]);
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if (act[j]) {
      double rj = h[j];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double Jjk = J[j * SMALL_M + k] + (j == k ? kappa : 0.0);
        if (act[k]) K[j][k] = Jjk; else { K[j][k] = 0.0; rj -= Jjk * delta[k]; }
      }
      r[j] = rj;
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) K[j][k] = (j == k) ? 1.0 : 0.0;
      r[j] = delta[j];
    }
  }
  // Cholesky K = L L^T (in place, lower triangle), all indices static.
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double dj = K[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= K[j][k] * K[j][k];
    dj = dj > 0.0 ? sqrt(dj) : sqrt(fmax(kappa, 1e-300));
    K[j][j] = dj;
    inv[j] = 1.0 / dj;                  // one division per pivot (a division is a long dependent chain)
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      double v = K[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= K[i][k] * K[j][k];
      K[i][j] = v * inv[j];
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double v = r[j];
#pragma unroll
    for (int k = 0; k < j; ++k) v -= K[j][k] * r[k];
    r[j] = v * inv[j];
  }
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {
    double v = r[j];
#pragma unroll
    for (int k = j + 1; k < M; ++k) v -= K[k][j] * r[k];
    r[j] = v * inv[j];
  }
#pragma unroll
  for (int j = 0; j < M; ++j) if (act[j]) delta[j] = r[j];
}

// Scaled KKT residual of the current iterate (stopping rule): active rows
// need |h_j| <= tol sigma_j, rows at lam_j = 0 need h_j <= tol sigma_j.
template <int M>
__device__ __forceinline__ double kkt_residual(const double* h, const double* lam, const double* scale, int eq) {
  double r = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double v = (((eq >> j) & 1) || lam[j] > 0.0) ? fabs(h[j]) : fmax(h[j], 0.0);
    r = fmax(r, v / scale[j]);
  }
  return r;
}

// The Newton control runs on one thread over register copies: every LDS
// value it needs is read up front (independent loads, one round trip) and
// every result written once.  Working on the LDS state directly would cost a
// dependent LDS round trip per access (several microseconds per step).

// Accept (lam, h, J) as the current iterate; decide to stop or start a line
// search.  Returns the next phase.
template <int M>
__device__ __forceinline__ int newton_accept(ShC& sh, const double (&lam)[M], const double (&h)[M],
                                             const double (&J)[M * SMALL_M]) {
  NewtonState& N = sh.N;
  double scale[M];
#pragma unroll
  for (int j = 0; j < M; ++j) scale[j] = sh.S.scale[j];
  const double kappa = sh.P.kappa, tol_n = sh.P.tol_n;
  const int ncp_mode = sh.P.ncp, max_newton = sh.P.max_newton, it = N.it;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    N.lam[j] = lam[j];
    N.h[j] = h[j];
#pragma unroll
    for (int k = 0; k < M; ++k) N.J[j * SMALL_M + k] = J[j * SMALL_M + k];
  }
  const int eq = sh.P.eq;
  const double res = kkt_residual<M>(h, lam, scale, eq);
  sh.res_inf = res;
  double phi[M], delta[M];
  bool act[M];
  ncp<M>(h, J, lam, kappa, ncp_mode, eq, phi, act);
  double p2 = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) p2 += phi[j] * phi[j];
  newton_direction<M>(h, J, lam, kappa, act, phi, ncp_mode, delta);
  if (res <= tol_n || it >= max_newton) {
    sh.outcome = res <= tol_n ? PGDTO_CONVERGED : PGDTO_MAXITER;
    // stated error: the step the float64 factor gives at the returned
    // multipliers (exact when the free pattern at the solution is the
    // current one), doubled
#pragma unroll
    for (int j = 0; j < M; ++j) {
      sh.lamf[j] = lam[j];
      sh.lerr[j] = 2.0 * fabs(delta[j]);
      sh.lslope[j] = J[j * SMALL_M + j] + kappa;
    }
    return PH_FINAL;
  }
  N.phi2 = p2;
  N.M0 = 0.5 * p2;
  N.gamma = 1.0;
  N.ls = 0;
  N.have_best = 0;
  N.it = it + 1;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    N.delta[j] = delta[j];
    N.trial[j] = ((eq >> j) & 1) ? lam[j] + delta[j] : fmax(lam[j] + delta[j], 0.0);
  }
  return PH_NEWTON;
}

// Line-search decision after evaluating the trial (tr, ht, Jt) (Appendix A.2:
// the largest gamma in (0,1] with the Armijo condition (c1) and the curvature
// condition (c2), searched by halving from 1).
template <int M>
__device__ __forceinline__ int newton_after_trial(ShC& sh, const double (&tr)[M], const double (&ht)[M],
                                                  const double (&Jt)[M * SMALL_M]) {
  NewtonState& N = sh.N;
  double delta[M], lam[M];
#pragma unroll
  for (int j = 0; j < M; ++j) { delta[j] = N.delta[j]; lam[j] = N.lam[j]; }
  const double kappa = sh.P.kappa, c1 = sh.P.c1, c2 = sh.P.c2;
  const int ncp_mode = sh.P.ncp, max_ls = sh.P.max_ls, eq = sh.P.eq;
  const double M0 = N.M0, phi2 = N.phi2, gamma = N.gamma;
  const int have_best = N.have_best, ls = N.ls + 1;
  double phi[M];
  bool act[M];
  ncp<M>(ht, Jt, tr, kappa, ncp_mode, eq, phi, act);
  double p2 = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) p2 += phi[j] * phi[j];
  const bool armijo = 0.5 * p2 <= M0 - c1 * gamma * phi2;
  // grad M(trial)^T Delta = Phi_t^T J_Phi(trial) Delta
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double row;
    if (act[j]) {
      row = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) row += (Jt[j * SMALL_M + k] + (j == k ? kappa : 0.0)) * delta[k];
    } else {
      row = (ncp_mode == PGDTO_NCP_PAPER) ? delta[j] : (Jt[j * SMALL_M + j] + kappa) * delta[j];
    }
    g += phi[j] * row;
  }
  const bool curv = g <= c2 * phi2;
  N.ls = ls;
  N.init = 0;
  if (armijo && !have_best) {
    N.have_best = 1;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      N.blam[j] = tr[j];
      N.bh[j] = ht[j];
#pragma unroll
      for (int k = 0; k < M; ++k) N.bJ[j * SMALL_M + k] = Jt[j * SMALL_M + k];
    }
  }
  if (armijo && curv) return newton_accept<M>(sh, tr, ht, Jt);
  if (ls >= max_ls) {
    if (have_best) {
      double bl[M], bh[M], bJ[M * SMALL_M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        bl[j] = N.blam[j];
        bh[j] = N.bh[j];
#pragma unroll
        for (int k = 0; k < M; ++k) bJ[j * SMALL_M + k] = N.bJ[j * SMALL_M + k];
      }
      return newton_accept<M>(sh, bl, bh, bJ);
    }
    return newton_accept<M>(sh, tr, ht, Jt);
  }
  const double gnew = 0.5 * gamma;
  N.gamma = gnew;
#pragma unroll
  for (int j = 0; j < M; ++j)
    N.trial[j] = ((eq >> j) & 1) ? lam[j] + gnew * delta[j] : fmax(lam[j] + gnew * delta[j], 0.0);
  return PH_NEWTON;
}

template <typename T, int M>
__device__ __forceinline__ void solve_coupled(ShC& sh, const Desc& d, int32_t* buf_end = nullptr) {
  constexpr int V = VT<T>::N;
  using C = CN<M>;
  const int tid = threadIdx.x;
  const int G = wg_num(d);
  const int wid = wg_id(d);
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  double kappa = d.kappa;           // the automatic penalty replaces it after the zero pass

  if (tid == 0) {
    sh.phase = d.pgd ? PH_PGD_R : PH_ZERO;
    sh.abort_flag = 0;
    sh.passes = 0;
    sh.path = 0;
    sh.outcome = PGDTO_INACTIVE;
    sh.nonfinite = 0;
    sh.s1passes = 0;
    sh.res_inf = 0.0;
    sh.pg.alpha = 0.0; sh.pg.beta = 0.0; sh.pg.used_fb = 0;
    sh.N.it = 0; sh.N.ls = 0; sh.N.init = 0; sh.N.have_best = 0;
    load_ctl(d, sh.P);
  }
  if (tid < M) {
    sh.bs[tid] = d.b[tid]; sh.lamf[tid] = 0.0; sh.N.lam1[tid] = 0.0;
    sh.lerr[tid] = 0.0; sh.lslope[tid] = 0.0; sh.amax[tid] = 0.0;
    sh.S.state[tid] = SEG_DONE; sh.S.lam[tid] = 0.0; sh.S.npass[tid] = 0; sh.S.width[tid] = 0.0;
    sh.S.outcome[tid] = PGDTO_INACTIVE; sh.S.scale[tid] = 1.0; sh.S.ssat[tid] = 0.0;
  }
  __syncthreads();

  int buf = d.buf0 & 1;
  const T* Arow[M];
#pragma unroll
  for (int j = 0; j < M; ++j) Arow[j] = (const T*)d.A + (int64_t)j * d.lda;
  T* X = (T*)d.x;
  const T* Y = d.pgd ? (const T*)d.x : (const T*)d.y;
  const T* sptr[M + 1];
  sptr[0] = Y;
#pragma unroll
  for (int j = 0; j < M; ++j) sptr[1 + j] = Arow[j];
  int ls_total = 0;

  int pass_no = 0;
  for (;;) {
    const int ph = sh.phase;
    double* pb = d.part + (size_t)buf * VMAX * TILES_PAD;
    const uint64_t t_pass0 = clk();
    trace_put(d, pass_no, 0, ((uint64_t)ph << 56) | (t_pass0 & 0x00ffffffffffffffull));
    int nv;
    uint64_t maxmask = 0;
    switch (ph) {
      case PH_PGD_R: nv = C::NV_R; maxmask = 1ull << 6; break;
      case PH_ZERO: nv = C::NV_ZERO; maxmask = (((1ull << M) - 1) << (2 * M)) | (((1ull << M) - 1) << (5 * M + 1)); break;
      case PH_STAGE1: nv = C::NV_S1; break;
      case PH_CHECK: nv = C::NV_CHECK; break;
      case PH_NEWTON: nv = C::NV_NEWTON; break;
      default: nv = C::NV_FINAL; break;
    }

    for (int tile = wid; tile < d.ntiles; tile += G) {
      const TileGeom g = tile_geom<T>(d, tile);
      if (ph == PH_PGD_R) {
        double acc[C::NV_R];
#pragma unroll
        for (int v = 0; v < C::NV_R; ++v) acc[v] = 0.0;
        const T* R = (const T*)d.rho; const T* RP = (const T*)d.rho_prev;
        const T* Gr = (const T*)d.grad; const T* GP = (const T*)d.grad_prev;
        for (int k = 0; k < g.nsweep; ++k) {
          int64_t e0; bool full; uint32_t mask;
          if (!slot<T>(g, k, e0, full, mask)) continue;
          T r[V], gr[V], rp[V], gp[V], a[M][V];
          ld_vec<T>(R, e0, d.n, full, r);
          ld_vec<T>(Gr, e0, d.n, full, gr);
          if (!d.zero_step) { ld_vec<T>(RP, e0, d.n, full, rp); ld_vec<T>(GP, e0, d.n, full, gp); }
#pragma unroll
          for (int j = 0; j < M; ++j) ld_vec<T>(Arow[j], e0, d.n, full, a[j]);
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            if (!d.zero_step) {
              const double sv = f64(r[q]) - f64(rp[q]), yv = f64(gr[q]) - f64(gp[q]);
              acc[0] = fma(sv, sv, acc[0]);
              acc[1] = fma(yv, yv, acc[1]);
              acc[2] = fma(sv, yv, acc[2]);
              acc[4] = fma(f64(gr[q]), yv, acc[4]);
              acc[5] = fma(f64(gp[q]), f64(gp[q]), acc[5]);
            }
            acc[3] = fma(f64(gr[q]), f64(gr[q]), acc[3]);
            acc[6] = fmax(acc[6], fabs(f64(gr[q])));
#pragma unroll
            for (int j = 0; j < M; ++j) acc[7 + j] = fma(f64(a[j][q]), f64(r[q]), acc[7 + j]);
          }
        }
        block_to_part<C::NV_R>(acc, nv, maxmask, sh.red, pb, tile);
      } else if (ph == PH_ZERO) {
        double acc[C::NV_ZERO];
#pragma unroll
        for (int v = 0; v < C::NV_ZERO; ++v) acc[v] = (v >= 2 * M && v < 3 * M) ? -INFINITY : 0.0;
        const T* R = (const T*)d.rho; const T* Gr = (const T*)d.grad; T* D = (T*)d.dir;
        const double beta = sh.pg.beta, step = d.omega * sh.pg.alpha;
        for (int k = 0; k < g.nsweep; ++k) {
          int64_t e0; bool full; uint32_t mask;
          if (!slot<T>(g, k, e0, full, mask)) continue;
          T yv[V], a[M][V];
#pragma unroll
          for (int j = 0; j < M; ++j) ld_vec<T>(Arow[j], e0, d.n, full, a[j]);
          if (d.pgd) {
            T r[V], gr[V], dp[V];
            ld_vec<T>(R, e0, d.n, full, r);
            ld_vec<T>(Gr, e0, d.n, full, gr);
            if (!d.zero_step) ld_vec<T>(D, e0, d.n, full, dp);
            T dn[V], rt[V];
#pragma unroll
            for (int q = 0; q < V; ++q) {
              const double dd = d.zero_step ? -f64(gr[q]) : fma(beta, f64(dp[q]), -f64(gr[q]));
              dn[q] = (T)dd;
              rt[q] = (T)fma(step, dd, f64(r[q]));
              yv[q] = rt[q];
            }
            st_vec<T>(D, e0, mask, full, dn);
            st_vec<T>(X, e0, mask, full, rt);
          } else {
            ld_vec<T>(Y, e0, d.n, full, yv);
          }
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            const double y = f64(yv[q]);
            const double x0 = clampd(y, lo, hi);
            const bool fr = (y >= lo && y <= hi);
            bool bad = !isfinite(y);
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const double av = f64(a[j][q]);
              acc[j] = fma(av, x0, acc[j]);
              if (fr) acc[M + j] = fma(av, av, acc[M + j]);
              if (av != 0.0) {
                const double bound = (av > 0.0) ? lo : hi;
                acc[2 * M + j] = fmax(acc[2 * M + j], breakpoint(y, av, bound));
                acc[3 * M + j] = fma(av, bound, acc[3 * M + j]);
              }
              acc[4 * M + j] += fabs(av);
              acc[5 * M + 1 + j] = fmax(acc[5 * M + 1 + j], fabs(av));
              bad |= !isfinite(av);
            }
            if (bad) acc[5 * M] += 1.0;
          }
        }
        block_to_part<C::NV_ZERO>(acc, nv, maxmask, sh.red, pb, tile);
      } else if (ph == PH_STAGE1) {
        double acc[C::NV_S1];
#pragma unroll
        for (int v = 0; v < C::NV_S1; ++v) acc[v] = 0.0;
        double lt[M][NT];
        bool on[M][NT];
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            lt[j][t] = sh.S.trial[j][t];
            on[j][t] = (sh.S.state[j] == SEG_SEARCH) && (lt[j][t] == lt[j][t]);
          }
        // row j alone at its trial lam_jt: a_j.clip(y - lam_jt a_j) and the slope sum_free a_j^2
        stream_tile<T, M + 1, C::U>(g, d.n, sptr, [&](const T (&b)[M + 1][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            const double yq = f64(b[0][q]);
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const double av = f64(b[1 + j][q]);
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                if (!on[j][t]) continue;
                const double z = fma(-lt[j][t], av, yq);
                acc[(j * NT + t) * 2] = fma(av, clampd(z, lo, hi), acc[(j * NT + t) * 2]);
                if (z >= lo && z <= hi) acc[(j * NT + t) * 2 + 1] = fma(av, av, acc[(j * NT + t) * 2 + 1]);
              }
            }
          }
        });
        block_to_part<C::NV_S1>(acc, nv, maxmask, sh.red, pb, tile);
      } else if (ph == PH_NEWTON) {
        // h and the upper triangle of A D A^T at the trial multiplier
        double acc[C::NV_NEWTON];
#pragma unroll
        for (int v = 0; v < C::NV_NEWTON; ++v) acc[v] = 0.0;
        double lamv[M];
#pragma unroll
        for (int j = 0; j < M; ++j) lamv[j] = sh.N.trial[j];
        stream_tile<T, M + 1, C::U>(g, d.n, sptr, [&](const T (&b)[M + 1][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            double z = f64(b[0][q]);
#pragma unroll
            for (int j = 0; j < M; ++j) z = fma(-lamv[j], f64(b[1 + j][q]), z);
            const double x = clampd(z, lo, hi);
            const bool fr = (z >= lo && z <= hi);
            double fa[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
              acc[j] = fma(f64(b[1 + j][q]), x, acc[j]);
              fa[j] = fr ? f64(b[1 + j][q]) : 0.0;
            }
            int p = M;
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
              for (int kk = j; kk < M; ++kk) { acc[p] = fma(fa[j], f64(b[1 + kk][q]), acc[p]); ++p; }
          }
        });
        block_to_part<C::NV_NEWTON>(acc, nv, maxmask, sh.red, pb, tile);
      } else if (ph == PH_CHECK) {
        // candidate sums a_k.x(lam_j* e_j) (+ the Newton sums at lam0 when fused)
        double acc[C::NV_CHECK];
#pragma unroll
        for (int v = 0; v < C::NV_CHECK; ++v) acc[v] = 0.0;
        double cand[M];
        bool con[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          cand[j] = sh.N.lam1[j];
          con[j] = cand[j] > 0.0;
        }
        stream_tile<T, M + 1, C::U>(g, d.n, sptr, [&](const T (&b)[M + 1][V], int64_t, uint32_t mask, bool) __attribute__((always_inline)) {
#pragma unroll
          for (int q = 0; q < V; ++q) {
            if (!(mask & (1u << q))) continue;
            const double yq = f64(b[0][q]);
#pragma unroll
            for (int j = 0; j < M; ++j) {
              if (!con[j]) continue;
              const double xc = clampd(fma(-cand[j], f64(b[1 + j][q]), yq), lo, hi);
#pragma unroll
              for (int kk = 0; kk < M; ++kk) acc[j * M + kk] = fma(f64(b[1 + kk][q]), xc, acc[j * M + kk]);
            }
            if constexpr (C::FUSE) {
              double z = yq;
#pragma unroll
              for (int j = 0; j < M; ++j) z = fma(-cand[j], f64(b[1 + j][q]), z);
              const double x = clampd(z, lo, hi);
              const bool fr = (z >= lo && z <= hi);
              double fa[M];
#pragma unroll
              for (int j = 0; j < M; ++j) {
                acc[M * M + j] = fma(f64(b[1 + j][q]), x, acc[M * M + j]);
                fa[j] = fr ? f64(b[1 + j][q]) : 0.0;
              }
              int p = M * M + M;
#pragma unroll
              for (int j = 0; j < M; ++j)
#pragma unroll
                for (int kk = j; kk < M; ++kk) { acc[p] = fma(fa[j], f64(b[1 + kk][q]), acc[p]); ++p; }
            }
          }
        });
        block_to_part<C::NV_CHECK>(acc, nv, maxmask, sh.red, pb, tile);
      } else {  // PH_FINAL
        double acc[C::NV_FINAL];
#pragma unroll
        for (int v = 0; v < C::NV_FINAL; ++v) acc[v] = 0.0;
        double lamv[M];
#pragma unroll
        for (int j = 0; j < M; ++j) lamv[j] = sh.lamf[j];
        const T* R = (const T*)d.rho;
        const int lane = tid & 63;
        // one slot ahead: y, the rows (and rho_t) of slot k + 1 are requested
        // before x of slot k is stored (x may alias y)
        constexpr int NF = M + 2;
        const T* fp[NF];
        fp[0] = Y;
#pragma unroll
        for (int j = 0; j < M; ++j) fp[1 + j] = Arow[j];
        fp[M + 1] = d.pgd ? R : Y;
        T nxt[1][NF][V];
        auto fetch = [&](int k) __attribute__((always_inline)) {
          int64_t e0 = d.n;                   // reads zeros
          if (k < g.nsweep) {
            bool full; uint32_t mask;
            if (!slot<T>(g, k, e0, full, mask)) e0 = d.n;
          }
          ld_slots<T, 1, NF>(fp, &e0, d.n, nxt);
        };
        fetch(0);
        for (int k = 0; k < g.nsweep; ++k) {
          int64_t e0; bool full; uint32_t mask;
          const bool any = slot<T>(g, k, e0, full, mask);
          T cur[NF][V];
#pragma unroll
          for (int q = 0; q < NF; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) cur[q][v] = nxt[0][q][v];
          fetch(k + 1);
          uint32_t bits = 0;
          if (any) {
            const T* yv = cur[0];
            const T (*a)[V] = &cur[1];
            const T* r = cur[M + 1];
            T xo[V];
#pragma unroll
            for (int q = 0; q < V; ++q) {
              double z = f64(yv[q]);
#pragma unroll
              for (int j = 0; j < M; ++j) z = fma(-lamv[j], f64(a[j][q]), z);
              xo[q] = (T)clampd(z, lo, hi);
              if (!(mask & (1u << q))) continue;
              const double xr = (double)xo[q];
#pragma unroll
              for (int j = 0; j < M; ++j) acc[j] = fma(f64(a[j][q]), xr, acc[j]);
              if (z >= lo && z <= hi) { acc[M] += 1.0; bits |= 1u << q; }
              if (d.pgd) {
                const double df = xr - f64(r[q]);
                acc[M + 1] = fma(df, df, acc[M + 1]);
                acc[M + 2] = fma(xr, xr, acc[M + 2]);
              }
              const double dy = xr - f64(yv[q]);          // distance of the projection
              acc[M + 3] = fma(dy, dy, acc[M + 3]);
            }
            st_vec<T>(X, e0, mask, full, xo);
          }
          if (d.free_mask) {
            constexpr int LPW = 32 / V;
            uint32_t w = any ? (bits << (uint32_t)(e0 & 31)) : 0u;
#pragma unroll
            for (int o = 1; o < LPW; o <<= 1) w |= (uint32_t)__shfl_xor((int)w, o, 64);
            // the tile's mask words were zeroed at entry: only words with set bits are written
            if (w != 0u && (lane % LPW) == 0) {
              const int64_t wi = e0 >> 5;
              const bool whole = (wi * 32 >= g.sstart) && (wi * 32 + 32 <= g.te);
              if (whole) d.free_mask[wi] = w;
              else atomicOr(&d.free_mask[wi], w);
            }
          }
        }
        block_to_part<C::NV_FINAL>(acc, nv, maxmask, sh.red, pb, tile);
      }
    }

    trace_put(d, pass_no, 1, clk());
    trace_wg(d, pass_no, t_pass0, clk());
    if (!grid_reduce(d, d.epoch0 + (uint64_t)pass_no + 1, pb, nv, maxmask, 1, sh.tot, &sh.abort_flag, pass_no)) break;
    trace_put(d, pass_no, 4, clk());

    // ---------------- control (identical in every workgroup)
    const double* t = sh.tot;
    if (ph == PH_PGD_R) {
      if (tid == 0) {
        pgd_scalars(d, t, sh.pg);
        sh.passes += 1;
        for (int j = 0; j < M; ++j) sh.bs[j] = d.b[j] + t[7 + j];
        sh.phase = PH_ZERO;
      }
    } else if (ph == PH_ZERO) {
      if (d.auto_tau > 0.0) {
        kappa = auto_kappa(d.auto_tau, &t[2 * M], 1, M);
        if (tid == 0) sh.P.kappa = kappa;     // the Newton control reads it from LDS
      }
      if (tid < M) {
        const int j = tid;
        double scale = t[4 * M + j] * fmax(fabs(lo), fabs(hi));
        if (!(scale > 0.0)) scale = 1.0;
        sh.S.scale[j] = scale;
        sh.amax[j] = t[5 * M + 1 + j];
        sh.asum[j] = t[4 * M + j];
        sh.S.slope[j] = t[M + j] + kappa;
        sh.N.h0[j] = t[j] - sh.bs[j];
        sh.S.ssat[j] = t[3 * M + j];
        if (d.stage1 && !d.eq_mask && !d.warm && t[5 * M] == 0.0) {
          search_init(sh.S, j, t[j] - sh.bs[j], t[M + j] + kappa, t[2 * M + j], t[3 * M + j], sh.bs[j], kappa,
                      scale, d.search, false);
        } else {
          sh.S.state[j] = SEG_DONE; sh.S.lam[j] = 0.0; sh.S.npass[j] = 0;
        }
      }
      __syncthreads();
      if (tid == 0) {
        sh.passes += 1;
        bool any_pos = false;     // some row needs a multiplier (equality rows: h(0) != 0)
        for (int j = 0; j < M; ++j) any_pos |= ((d.eq_mask >> j) & 1) ? (sh.N.h0[j] != 0.0) : (sh.N.h0[j] > 0.0);
        if (t[5 * M] > 0.0) {
          sh.nonfinite = 1;
          sh.outcome = PGDTO_NONFINITE;
          sh.phase = PH_FINAL;
        } else if (!any_pos) {
          sh.outcome = PGDTO_INACTIVE;
          sh.path = 0;
          sh.phase = PH_FINAL;
        } else if (!d.stage1 || d.eq_mask || d.warm) {
          // Stage 1 tests single active rows; equality rows are always
          // active, so with any of them Newton starts at lam = 0; a warm
          // start begins Newton at the given multipliers
          sh.path = 3;
          for (int j = 0; j < M; ++j) sh.N.trial[j] = d.warm ? d.lam0[j] : 0.0;
          sh.N.init = 1;
          sh.phase = PH_NEWTON;
        } else {
          int any = 0;
          for (int j = 0; j < M; ++j) any |= (sh.S.state[j] == SEG_SEARCH);
          sh.phase = any ? PH_STAGE1 : PH_CHECK;
          if (!any) for (int j = 0; j < M; ++j) sh.N.lam1[j] = sh.S.lam[j];
        }
      }
    } else if (ph == PH_STAGE1) {
      if (tid < M && sh.S.state[tid] == SEG_SEARCH) {
        const int j = tid;
        search_update(sh.S, j, t[(j * NT + 0) * 2], t[(j * NT + 1) * 2], t[(j * NT + 0) * 2 + 1],
                      t[(j * NT + 1) * 2 + 1], sh.bs[j], kappa, d.tol_n, d.tol_b, d.max_search, d.search, false);
      }
      __syncthreads();
      if (tid == 0) {
        sh.passes += 1;
        sh.s1passes += 1;
        int any = 0;
        for (int j = 0; j < M; ++j) any |= (sh.S.state[j] == SEG_SEARCH);
        if (!any) {
          for (int j = 0; j < M; ++j) sh.N.lam1[j] = sh.S.lam[j];
          sh.phase = PH_CHECK;
        }
      }
    } else if (ph == PH_CHECK) {
      if (tid == 0) {
        sh.passes += 1;
        int found = -1;
        for (int j = 0; j < M && found < 0; ++j) {
          if (!(sh.N.lam1[j] > 0.0)) continue;
          bool ok = true;
          for (int k = 0; k < M; ++k) {
            const double hk = t[j * M + k] - sh.bs[k] - (k == j ? kappa * sh.N.lam1[j] : 0.0);
            if (hk > d.tol_n * sh.S.scale[k]) { ok = false; break; }
          }
          if (ok) found = j;
        }
        if (found >= 0) {
          for (int j = 0; j < M; ++j) {
            sh.lamf[j] = (j == found) ? sh.N.lam1[j] : 0.0;
            sh.lerr[j] = (j == found) ? sh.S.err[j] : 0.0;
            sh.lslope[j] = sh.S.slope[j];
          }
          sh.path = 2;
          sh.outcome = PGDTO_CONVERGED;
          sh.phase = PH_FINAL;
        } else {
          sh.path = 3;
          if (C::FUSE) {
            double l1[M], ht[M], Jt[M * SMALL_M];
#pragma unroll
            for (int j = 0; j < M; ++j) l1[j] = sh.N.lam1[j];
#pragma unroll
            for (int j = 0; j < M; ++j) ht[j] = t[M * M + j] - sh.bs[j] - kappa * l1[j];
            unpack_J<M>(&t[M * M + M], Jt);
            sh.phase = newton_accept<M>(sh, l1, ht, Jt);
          } else {
            for (int j = 0; j < M; ++j) sh.N.trial[j] = sh.N.lam1[j];
            sh.N.init = 1;
            sh.phase = PH_NEWTON;
          }
        }
      }
    } else if (ph == PH_NEWTON) {
      if (tid == 0) {
        sh.passes += 1;
        ls_total += 1;
        // the evaluated trial, its h and J, in registers
        double tr[M], ht[M], Jt[M * SMALL_M];
#pragma unroll
        for (int j = 0; j < M; ++j) tr[j] = sh.N.trial[j];
#pragma unroll
        for (int j = 0; j < M; ++j) ht[j] = t[j] - sh.bs[j] - kappa * tr[j];
        unpack_J<M>(&t[M], Jt);
        if (sh.N.init) {
          sh.N.init = 0;
          sh.phase = newton_accept<M>(sh, tr, ht, Jt);
        } else {
          sh.phase = newton_after_trial<M>(sh, tr, ht, Jt);
        }
      }
    } else {  // PH_FINAL
      if (wid == 0) {
        pgdto_result* R = d.pgd ? &((pgdto_pgd_out*)d.result)->proj : (pgdto_result*)d.result;
        if (tid < M) {
          const int j = tid;
          const bool eqj = (d.eq_mask >> j) & 1ull;
          const double lamj = sh.lamf[j];
          R->lambda[j] = lamj;
          R->resid[j] = t[j] - sh.bs[j];
          R->slack[j] = kappa * lamj;
          // equality rows are always active (Sec. 3.2): converged with a
          // multiplier of either sign, infeasible when b_j lies outside the
          // range of a_j.x over the box [ssat_j, ssat_j + sum |a_j| (hi - lo)]
          int o = (eqj || lamj > 0.0) ? PGDTO_CONVERGED : PGDTO_INACTIVE;
          if (sh.S.ssat[j] - sh.bs[j] > 0.0) o = PGDTO_INFEASIBLE;
          if (eqj && sh.bs[j] - (sh.S.ssat[j] + sh.asum[j] * (hi - lo)) > 0.0) o = PGDTO_INFEASIBLE;
          if (sh.outcome == PGDTO_MAXITER || sh.outcome == PGDTO_NONFINITE) o = sh.outcome;
          R->row_outcome[j] = o;
          const double le = sh.nonfinite ? INFINITY : lam_error(lamj, sh.lerr[j], sh.S.scale[j], sh.lslope[j]);
          R->lambda_err[j] = le;
          const double h = t[j] - sh.bs[j] - kappa * lamj;
          // per-row values for the summary below, through LDS
          sh.red[j] = ((eqj || lamj != 0.0) ? fabs(h) : fmax(h, 0.0)) / sh.S.scale[j];
          sh.red[SMALL_M + j] = le;
          sh.red[2 * SMALL_M + j] = (double)o;
        }
        __syncthreads();
        if (tid == 0) {
          int worst = sh.outcome;
          double rmax = 0.0, xerr = 0.0;
          for (int j = 0; j < M; ++j) {
            if ((int)sh.red[2 * SMALL_M + j] == PGDTO_INFEASIBLE && severity(PGDTO_INFEASIBLE) > severity(worst))
              worst = PGDTO_INFEASIBLE;
            rmax = fmax(rmax, sh.red[j]);
            xerr += sh.amax[j] * sh.red[SMALL_M + j];
          }
          R->outcome = worst;
          R->error = 0;
          R->path = sh.path;
          R->passes = sh.passes + 1;
          int np = 0;
          for (int j = 0; j < M; ++j) np = max(np, sh.S.npass[j]);
          R->iters_search = np;
          R->iters_newton = sh.N.it;
          R->iters_ls = ls_total;
          R->m = M;
          R->n_free = (int64_t)t[M];
          R->res_inf = rmax;
          R->n_compact = -1;                       // the coupled path does not compact
          R->passes_compacted = 0;
          R->dist2 = t[M + 3];
          R->x_err = xerr + half_ulp(fmax(fabs(lo), fabs(hi)), sizeof(T) == 4);
          double wmax = 0.0;
          for (int j = 0; j < M; ++j) wmax = fmax(wmax, sh.S.width[j]);
          R->lambda_width = wmax;
          R->kappa = kappa;
          if (d.pgd) {
            pgdto_pgd_out* P = (pgdto_pgd_out*)d.result;
            P->alpha = sh.pg.alpha;
            P->beta = sh.pg.beta;
            P->used_fallback = sh.pg.used_fb;
            P->rel_change = (t[M + 2] > 0.0) ? sqrt(t[M + 1]) / sqrt(t[M + 2]) : INFINITY;
            P->converged = (P->rel_change <= d.tol_stop) ? 1 : 0;
          }
        }
      }
      if (tid == 0) sh.phase = PH_DONE;
    }
    __syncthreads();
    trace_put(d, pass_no, 5, clk());
    ++pass_no;
    buf ^= 1;
    if (sh.phase == PH_DONE) break;
  }
  int32_t* errp = nullptr;
  if (d.result) errp = d.pgd ? &((pgdto_pgd_out*)d.result)->proj.error : &((pgdto_result*)d.result)->error;
  report_error(d, errp);
  if (buf_end && threadIdx.x == 0) *buf_end = buf;     // the next instance of a batch slot starts there
}

template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void k_solve_coupled(const Desc) {
  __shared__ ShC sh;
  __shared__ Desc sd;
  __shared__ int32_t late;
  load_desc(sd);
  if (!enter_launch(sd, &late)) return;
  clear_mask_tiles<T>(sd);
  solve_coupled<T, M>(sh, sd);
}

// ================================================================== server kernel
// Continuous batching: slot s owns workgroups [s * W, (s + 1) * W) of one
// long-running launch.  Its first workgroup claims the next published job
// (one compare-and-swap on the device-wide head counter), broadcasts it to
// the slot, every workgroup of the slot copies the job's descriptor, clears
// the free-mask words of its tiles and runs the same solver as a one-instance
// launch on W workgroups, with the slot's own partial sums and barrier words.
// Jobs are projections or Algorithm 3 steps.  Results are bitwise those of a
// one-instance launch: the reduction order follows the tiles, which depend
// only on n and the dtype.  A slot leaves
// when the host sets shutdown and no job is left, or after idle_spins polls
// without a job (the host launches the kernel again when new work comes).
// float32 streams only.

union ShSrv {
  Sh1D s1;
  ShC sc;
};

// The server's shared state lives at namespace scope so that each solver
// variant can be a separate (not inlined) function that still addresses LDS
// directly: the register allocation of every variant then stays that of its
// one-instance kernel instead of the maximum over all variants of one huge
// function.
__shared__ ShSrv srv_sh;
__shared__ Desc srv_sd;

__shared__ int32_t srv_buf_end;     // partial-sum buffer after the last solve
template <bool EQ, bool CP, bool NT = false>
__device__ __noinline__ void srv_solve_1d() { solve_1d<float, EQ, CP, 2, NT>(srv_sh.s1, srv_sd, &srv_buf_end); }
template <int M>
__device__ __noinline__ void srv_solve_coupled() { solve_coupled<float, M>(srv_sh.sc, srv_sd, &srv_buf_end); }


__global__ __launch_bounds__(BLOCK) void k_server(const SrvArgs) {
  __shared__ SrvArgs a;
  Desc& sd = srv_sd;
  __shared__ int64_t job;
  __shared__ int32_t leave;
  {
    const uint32_t* src = (const uint32_t*)__builtin_amdgcn_kernarg_segment_ptr();
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
    for (int i = threadIdx.x; i < (int)(sizeof(SrvArgs) / 4); i += BLOCK) dst[i] = src[i];
    __syncthreads();
  }
  const int W = a.wg_per_slot;
  const int slot = (int)blockIdx.x / W;
  const int vb = (int)blockIdx.x - slot * W;
  uint64_t* sw = a.slot_words + (size_t)slot * 16;
  int32_t nbuf = 0;          // partial-sum buffer of the slot's next pass
  for (uint64_t r = 1;; ++r) {
    const uint64_t seq = a.round0 + r;
    if (threadIdx.x == 0) {
      int64_t j = -1;
      int out = 0;
      if (vb == 0) {
        uint32_t spins = 0;
        for (;;) {
          const uint64_t tail = __hip_atomic_load(&a.ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          uint64_t h = __hip_atomic_load(a.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (h < tail) {
            if (__hip_atomic_compare_exchange_strong(a.head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
              j = (int64_t)h;
              break;
            }
            continue;
          }
          if (__hip_atomic_load(&a.ctl->shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0 ||
              ++spins > a.idle_spins) {
            out = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(32);
        }
        __hip_atomic_store(sw + 1, out ? SRV_LEAVE : (uint64_t)j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sw, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        // bounded: well beyond the master's idle time
        uint32_t spins = 0;
        while (__hip_atomic_load(sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < seq) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins > 16u * a.idle_spins + SPIN_LIMIT) { out = 1; break; }
        }
        if (!out) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          const uint64_t v = __hip_atomic_load(sw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v == SRV_LEAVE) out = 1; else j = (int64_t)v;
        }
      }
      job = j;
      leave = out;
    }
    __syncthreads();
    if (leave) return;
    const int64_t jb = job;
    const int q = (int)(jb % a.qcap);
    {
      // the job descriptor (pinned host memory, published before tail)
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a.jobs + q);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sd);
      for (int i = threadIdx.x; i < (int)(sizeof(Desc) / 4); i += BLOCK)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();
      if (threadIdx.x == 0) {
        sd.wg_base = slot * W;
        sd.wg_count = W;
        sd.part = a.part + (size_t)slot * a.part_stride;
        sd.sync = a.sync + (size_t)slot * a.sync_stride;
        sd.result = sd.pgd ? (void*)(a.results + q) : (void*)&a.results[q].proj;
        sd.trace = nullptr;
        // every workgroup of the slot reduces the pass partials itself; the
        // two buffers keep alternating across the slot's jobs (a workgroup
        // that starts the next job cannot overwrite partials another
        // workgroup of the slot is still reading)
        sd.allred = W <= ALLRED_MAX_WG ? 1 : 0;
        sd.buf0 = nbuf;
      }
      __syncthreads();
    }
    clear_mask_tiles<float>(sd);
    if (sd.kind == PGDTO_COUPLED) {
      switch (sd.m) {
        case 1: srv_solve_coupled<1>(); break;
        case 2: srv_solve_coupled<2>(); break;
        case 3: srv_solve_coupled<3>(); break;
        case 4: srv_solve_coupled<4>(); break;
        case 5: srv_solve_coupled<5>(); break;
        case 6: srv_solve_coupled<6>(); break;
        case 7: srv_solve_coupled<7>(); break;
        default: srv_solve_coupled<8>(); break;
      }
    } else {
      const bool cp = srv_sd.compact && srv_sd.cbuf;
      if (srv_sd.eq_mask) {
        if (cp) srv_solve_1d<true, true>(); else srv_solve_1d<true, false>();
      } else {
        if (cp) srv_solve_1d<false, true>(); else srv_solve_1d<false, false>();
      }
    }
    __syncthreads();
    nbuf = srv_buf_end;
    if (vb == 0 && threadIdx.x == 0) {
      // the result (written by this workgroup) before the completion word
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      __hip_atomic_store(a.done + q, (uint64_t)jb + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ================================================================== batch kernel
// Many instances in one launch: slot s owns workgroups [s * W, (s + 1) * W)
// and solves instances s, s + slots, s + 2 slots, ... of the list in order,
// with the same solver and the same per-slot workspace as the server.  The
// k-th instance of a slot takes barrier epochs from epoch_base + (k << 16),
// above every flag its predecessors left.  A workgroup that finishes an
// instance early starts the next one at once: the next instance's first
// totals need this workgroup's flag, so no workgroup of the slot can still
// be reading the previous instance's totals when they are overwritten.
// float32 streams only.
__global__ __launch_bounds__(BLOCK) void k_batch(const BatchArgs) {
  __shared__ BatchArgs a;
  Desc& sd = srv_sd;
  {
    const uint32_t* src = (const uint32_t*)__builtin_amdgcn_kernarg_segment_ptr();
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
    for (int i = threadIdx.x; i < (int)(sizeof(BatchArgs) / 4); i += BLOCK) dst[i] = src[i];
    __syncthreads();
  }
  const int W = a.wg_per_slot;
  const int slot = (int)blockIdx.x / W;
  if (slot >= a.slots) return;
  int32_t nbuf = 0;          // partial-sum buffer of the slot's next pass
  for (int k = 0;; ++k) {
    const int64_t i = (int64_t)slot + (int64_t)k * a.slots;
    if (i >= a.count) return;
    {
      // the instance's descriptor (pinned host memory, written before the launch)
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a.jobs + i);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sd);
      for (int w = threadIdx.x; w < (int)(sizeof(Desc) / 4); w += BLOCK)
        dst[w] = __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();
      if (threadIdx.x == 0) {
        sd.wg_base = slot * W;
        sd.wg_count = W;
        sd.part = a.part + (size_t)slot * a.part_stride;
        sd.sync = a.sync + (size_t)slot * a.sync_stride;
        sd.epoch0 = a.epoch_base + ((uint64_t)k << BATCH_JOB_SHIFT);
        sd.pgd = a.is_pgd;
        sd.result = a.is_pgd ? (void*)((pgdto_pgd_out*)a.results + i) : (void*)((pgdto_result*)a.results + i);
        sd.trace = nullptr;
        // every workgroup of the slot reduces the pass partials itself; the
        // two buffers keep alternating across the slot's instances
        sd.allred = W <= ALLRED_MAX_WG ? 1 : 0;
        sd.buf0 = nbuf;
      }
      __syncthreads();
    }
    clear_mask_tiles<float>(sd);
    if (sd.kind == PGDTO_COUPLED) {
      switch (sd.m) {
        case 1: srv_solve_coupled<1>(); break;
        case 2: srv_solve_coupled<2>(); break;
        case 3: srv_solve_coupled<3>(); break;
        case 4: srv_solve_coupled<4>(); break;
        case 5: srv_solve_coupled<5>(); break;
        case 6: srv_solve_coupled<6>(); break;
        case 7: srv_solve_coupled<7>(); break;
        default: srv_solve_coupled<8>(); break;
      }
    } else {
      // Algorithm 3 steps stream five arrays per instance: non-temporal loads
      // (the compaction variant re-reads the pairs it keeps: ordinary loads)
      const bool cp = srv_sd.compact && srv_sd.cbuf;
      const bool nt = a.is_pgd && !cp;
      if (srv_sd.eq_mask) {
        if (cp) srv_solve_1d<true, true>(); else if (nt) srv_solve_1d<true, false, true>(); else srv_solve_1d<true, false>();
      } else {
        if (cp) srv_solve_1d<false, true>(); else if (nt) srv_solve_1d<false, false, true>(); else srv_solve_1d<false, false>();
      }
    }
    __syncthreads();
    nbuf = srv_buf_end;
  }
}

// Marks a result as failed (used by the host after a failed launch).
__global__ void k_mark_error(void* result, int is_pgd) {
  if (threadIdx.x == 0 && result) {
    pgdto_result* R = is_pgd ? &((pgdto_pgd_out*)result)->proj : (pgdto_result*)result;
    R->error = PGDTO_ERR_HIP;
  }
}

// ------------------------------------------------------------------ launchers

template <typename T>
static const void* coupled_fn(int m) {
  switch (m) {
    case 1: return (const void*)k_solve_coupled<T, 1>;
    case 2: return (const void*)k_solve_coupled<T, 2>;
    case 3: return (const void*)k_solve_coupled<T, 3>;
    case 4: return (const void*)k_solve_coupled<T, 4>;
    case 5: return (const void*)k_solve_coupled<T, 5>;
    case 6: return (const void*)k_solve_coupled<T, 6>;
    case 7: return (const void*)k_solve_coupled<T, 7>;
    default: return (const void*)k_solve_coupled<T, 8>;
  }
}

template <typename T>
static const void* solve_1d_fn(bool eq, bool cp) {
  if (eq) return cp ? (const void*)k_solve_1d<T, true, true> : (const void*)k_solve_1d<T, true, false>;
  return cp ? (const void*)k_solve_1d<T, false, true> : (const void*)k_solve_1d<T, false, false>;
}

static const void* kernel_fn(int kind, int dtype, int m, bool eq, bool cp) {
  if (kind == PGDTO_COUPLED && m > SMALL_M) return wide_fn(m);
  if (kind == PGDTO_COUPLED) return dtype == PGDTO_F32 ? coupled_fn<float>(m) : coupled_fn<double>(m);
  return dtype == PGDTO_F32 ? solve_1d_fn<float>(eq, cp) : solve_1d_fn<double>(eq, cp);
}

int max_coresident(int kind, int dtype, int m, int device) {
  int nb = 0, ncu = 0;
  // the plain and the compaction instantiations of a kernel fit alike (both
  // take at most 256 VGPRs); the smaller count of the two is used
  int nb2 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_fn(kind, dtype, m, false, false), BLOCK, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, kernel_fn(kind, dtype, m, false, true), BLOCK, 0) != hipSuccess)
    return 0;
  nb = nb < nb2 ? nb : nb2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return nb * ncu;
}

hipError_t launch_solve(const Desc& d, int grid, hipStream_t stream, bool cooperative) {
  Desc copy = d;
  void* args[] = {&copy};
  const void* fn = kernel_fn(d.kind, d.dtype, d.m, d.eq_mask != 0, d.compact && d.cbuf);
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BLOCK), args, 0, stream);
  return hipLaunchKernel(fn, dim3(grid), dim3(BLOCK), args, 0, stream);
}

hipError_t launch_server(const SrvArgs& a, hipStream_t stream) {
  SrvArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_server, dim3(a.slots * a.wg_per_slot), dim3(BLOCK), args, 0, stream);
}

int server_coresident(int device) {
  int nb = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_server, BLOCK, 0) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return nb * ncu;
}

hipError_t launch_batch(const BatchArgs& a, hipStream_t stream) {
  BatchArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel((const void*)k_batch, dim3(a.slots * a.wg_per_slot), dim3(BLOCK), args, 0, stream);
}

int batch_coresident(int device) {
  int nb = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_batch, BLOCK, 0) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return nb * ncu;
}

hipError_t launch_mark_error(void* result, int is_pgd, hipStream_t stream) {
  hipLaunchKernelGGL(k_mark_error, dim3(1), dim3(64), 0, stream, result, is_pgd);
  return hipGetLastError();
}

// ------------------------------------------------------------------ static scratch
// Workspace of pgdto_project_noalloc: the per-tile partial sums followed by
// the barrier and arrival-door words, laid out as in a context.  One copy per
// GPU, resident from module load to process end.  In host code `scratch`
// names a host-side stand-in; its device address on the current GPU comes
// from hipGetSymbolAddress, once per device, and only that address is ever
// passed to a kernel.
constexpr size_t NOALLOC_WORDS = (size_t)PART_DOUBLES + SYNC_WORDS;
static_assert(NOALLOC_WORDS * sizeof(uint64_t) == PGDTO_NOALLOC_SCRATCH_BYTES, "scratch size in pgdto.h");
static __device__ __align__(256) uint64_t scratch[NOALLOC_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;

struct NoallocDevice {
  uint64_t* ptr = nullptr;                  // device address of `scratch` on this GPU
  int cap[2][2][PGDTO_MAX_M + 1] = {};      // co-resident workgroups per kernel
};
static NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];
static std::mutex g_noalloc_mu;

// Clears the scratch words (the first call on a device).  A kernel rather
// than a memset, so that a call captured into a HIP graph records a kernel node.
__global__ __launch_bounds__(256) void k_clear_words(uint64_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace pgdto

extern "C" int pgdto_project_noalloc(const pgdto_problem* prob, const pgdto_params* params, pgdto_result* result_dev,
                                     void* stream) {
  using namespace pgdto;
  if (!prob || !result_dev) return PGDTO_ERR_ARG;
  pgdto_params tmp;
  if (!params) {
    pgdto_params_default(&tmp);
    params = &tmp;
  }
  Desc d;
  const int st = build_desc(prob, params, true, d);
  if (st != PGDTO_OK) return st;
  // the partial-sum table holds TILES_PAD tiles of VMAX values (sized for
  // SMALL_M coupled rows), the totals at most TOT_MAX values; more coupled
  // rows need the much larger workspace of the wide kernel
  if (d.ntiles > TILES_PAD || (d.kind == PGDTO_COUPLED && d.m > SMALL_M) || d.nseg * 9 > TOT_MAX)
    return PGDTO_ERR_SCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return PGDTO_ERR_HIP;
  const hipStream_t s = (hipStream_t)stream;
  uint64_t* ws = nullptr;
  bool first = false;
  int grid = 0;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoallocDevice& D = g_noalloc[dev];
    if (!D.ptr) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PGDTO_ERR_HIP;
      D.ptr = (uint64_t*)p;
      first = true;
    }
    ws = D.ptr;
    const int ki = d.kind == PGDTO_COUPLED ? 1 : 0;
    int& cap = D.cap[ki][d.dtype][ki ? d.m : 0];
    if (cap == 0) cap = max_coresident(d.kind, d.dtype, d.m, dev);
    if (cap <= 0) return PGDTO_ERR_HIP;
    grid = d.ntiles < cap ? d.ntiles : cap;
    if (grid < 1) grid = 1;
  }
  if (first) {
    hipLaunchKernelGGL(k_clear_words, dim3(256), dim3(256), 0, s, ws, NOALLOC_WORDS);
    if (hipGetLastError() != hipSuccess) {
      std::lock_guard<std::mutex> lock(g_noalloc_mu);
      g_noalloc[dev].ptr = nullptr;        // clear again on the next call
      return PGDTO_ERR_HIP;
    }
  }
  d.part = (double*)ws;
  d.sync = ws + PART_DOUBLES;
  d.epoch0 = 0;                            // replaced on the device by the door's generation
  d.trace = nullptr;
  d.result = result_dev;
  d.pgd = 0;
  d.wg_base = 0;
  d.wg_count = grid;
  d.door_wait = DOOR_WAIT_DEFAULT;
  d.allred = grid <= ALLRED_MAX_WG ? 1 : 0;   // as the other one-instance launches
  d.buf0 = 0;
  if (launch_solve(d, grid, s, false) != hipSuccess) {
    (void)hipGetLastError();
    (void)launch_mark_error(result_dev, 0, s);
    return PGDTO_ERR_HIP;
  }
  return PGDTO_OK;
}
