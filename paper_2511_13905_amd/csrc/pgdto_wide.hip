// Coupled rows beyond SMALL_M: Algorithm 2 for up to PGDTO_MAX_M dense rows.
//
// The small coupled kernel keeps every partial sum of a thread in registers;
// at m = 32..64 the Newton pass has m + m(m+1)/2 sums (eq. h and the
// Jacobian of eq. reg_jacobian, J = A D A^T with D the free indicator), about
// m^2 flops per element against 4 (m + 1) bytes: past the float32 ridge of
// the chip at m ~ 40.  This kernel therefore
//
//  * lays a wave's data out as the matrix cores want it: lane (r, g), r =
//    lane % 16, g = lane / 16, holds rows 16 bj + r (bj < MB) of 8
//    elements of a 32-element chunk (two float4s, see elem_off).  That is
//    both the A operand (row i = r, reduction index k = g) and the B
//    operand (k = g, column j = r) of
//    v_mfma_f32_16x16x4_f32, so the free-masked tile F = D^(1/2) A of 32
//    elements feeds 8 k-steps of F F^T on the MB (MB + 1) / 2 upper-triangle
//    16 x 16 blocks with no data movement;
//  * computes z = y - A^T lam in float64 as per-lane partial dot products
//    over the lane's rows, added over the 16 lanes of a row group with DPP
//    row rotations (every lane of the group gets the same bits), and h in
//    float64 per row;
//  * checks the Stage-1 candidates (m^2 sums a_k . x(lam_j e_j), compared
//    against a tolerance relative to sigma_k, so float64 throughout) with
//    v_mfma_f64_16x16x4_f64 on at most 16 candidates per pass;
//  * reduces the per-tile partials over the grid in two steps -- every
//    workgroup publishes its tiles' values, then every workgroup sums a slice
//    of the values over all tiles in a fixed order -- because the 2144 sums
//    of a Newton pass at m = 64 are far too many for one workgroup;
//  * runs the float64 control on workgroup 0 only (continuous NCP, a
//    workgroup-parallel LDL^T factorisation of the active block of
//    A D A^T + kappa I, the Armijo/curvature line search of Appendix A.2) and
//    broadcasts the next pass's command (phase and multipliers).
//
// Reduction orders depend only on n, m and the dtype, never on the grid, so
// results are bitwise reproducible at any grid size.  Float32 streams,
// projections only (the Algorithm 3 step and the batch and serving routes
// stay with m <= SMALL_M).
//
// Lane-layout facts used below (16x16x4 MFMA, checked on the device): A
// operand lane l holds A[l % 16][l / 16] and B operand lane l holds
// B[l / 16][l % 16], for f32 and f64 alike; output register q of lane l is
// D[4 (l / 16) + q][l % 16] for f32 but D[l / 16 + 4 q][l % 16] for f64.

#include "pgdto_device.h"

namespace pgdto {

typedef float wf32x4 __attribute__((ext_vector_type(4)));
typedef double wf64x4 __attribute__((ext_vector_type(4)));

constexpr int WCH = 32;      // elements per wave and chunk (one free-mask word)
constexpr int WSL = 8;       // elements per lane and chunk
constexpr int REP_PH = 1, REP_AUX = 2, REP_PAY = 4;   // words of a command replica after the go word
constexpr int WNREP = 32;    // command replicas in use (of NREP): 8 workgroups read each at a full grid

// The 8 elements of lane group g within a chunk: e0 + 4 g + s for s < 4 and
// e0 + 16 + 4 g + (s - 4) for s >= 4, so that each load instruction covers 64
// contiguous bytes of each of 16 rows (the groups' float4s side by side).
__device__ __forceinline__ int elem_off(int g, int s) { return s < 4 ? 4 * g + s : 12 + 4 * g + s; }

template <int MB> struct WN {
  static constexpr int NB = MB * (MB + 1) / 2;   // upper-triangle 16 x 16 blocks of J
};

// Index of J[j][k], j <= k, in the packed upper triangle (row-major, the
// layout of the small kernel's Newton sums).
__device__ __forceinline__ int pk(int j, int k, int m) { return j * m - (j * (j - 1)) / 2 + (k - j); }
__device__ __forceinline__ int pks(int j, int k, int m) { return j <= k ? pk(j, k, m) : pk(k, j, m); }

// Block bi of the upper triangle (row-major over bj <= bk).
template <int MB>
__device__ __forceinline__ void block_rc(int bi, int& bj, int& bk) {
  int q = bi, j = 0;
  while (q >= MB - j) { q -= MB - j; ++j; }
  bj = j;
  bk = j + q;
}

// Sum over the 16 lanes of a row group by DPP row rotations; the result is
// bitwise the same in all 16 lanes (each step adds two values that the
// partner lane adds in the other order).
template <int K>
__device__ __forceinline__ double row_ror(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x120 + K, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x120 + K, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}

// A wave-uniform lane's double, through two scalar reads.
__device__ __forceinline__ double lane_value(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------------------ workspace
struct WSync {
  double* part;      // [WTILES][WV_PAD] per-tile partial sums
  double* tot;       // [WV_PAD] totals of the pass
  double* best;      // [WNJ] Jacobian of the best Armijo trial (workgroup 0)
  uint64_t* flags;   // [GMAX][FLAG_STRIDE]
  uint64_t* rep;     // [NREP][WREP]: go word, phase, aux, payload
  uint64_t* err;     // the context's error line
};

__device__ __forceinline__ WSync wide_words(const Desc& d) {
  WSync w;
  w.part = d.wide + WIDE_PART;
  w.tot = d.wide + WIDE_TOT;
  w.best = d.wide + WIDE_BEST;
  w.flags = (uint64_t*)(d.wide + WIDE_FLAGS);
  w.rep = (uint64_t*)(d.wide + WIDE_REP);
  w.err = sync_words(d).err;
  return w;
}

// ------------------------------------------------------------------ shared state
struct ShW {
  double tot[WV_PAD];          // totals of the pass (workgroup 0); the LDL^T factor overwrites the J part
  double pay[2 * WM];          // command payload: Stage 1 trials [2j + t]; check: lam of the candidates
                               // [0, 16), their rows [16, 32); Newton trial / final multipliers [j]
  int32_t ph, aux, abort_flag, np;
  Search S;
  double bs[WM], lamf[WM], lerr[WM], lslope[WM], amax[WM], asum[WM];
  double lam[WM], h[WM], delta[WM], blam[WM], bh[WM], lam1[WM], h0[WM], htr[WM];
  double phi[WM], rowv[WM], rhs[WM], dv[WM], diagc[WM];
  double colbuf[2][WM];
  int32_t act[WM], sidx[WM];
  uint64_t eq;
  double kappa, tol_n, tol_b, c1, c2, phi2, M0, gamma, res_inf, p2;
  int32_t max_newton, max_ls, max_search, ncp, search;
  int32_t have_best, ls, it, init, passes, path, outcome, nonfinite, s1passes, ls_total, cnext, decision;
  uint64_t tmark[2];           // trace: totals in LDS, Newton direction solved
  union {
    float f[NWAVE * 2 * 256];  // two J blocks per round
    double d[NWAVE * 256];     // one float64 block per round, per-row values, scalars
  } red;
};

// ------------------------------------------------------------------ streaming

// Streams the chunks of a tile: wave w takes the whole chunks w, w + NWAVE,
// ... with the loads of its next chunk in flight while the current one is
// used (two register buffers in turn), then the wave whose turn it is takes
// the ragged last chunk, if any.  f(y, a, e0, whole): y[s], a[bj][s] of this
// lane for element e0 + elem_off(g, s) (zeros past the tile end and for rows
// >= m), e0 the chunk's first element, whole = all 32 elements inside the tile.
template <int MB, class F>
__device__ __forceinline__ void wide_chunks(const Desc& d, int64_t ts, int64_t te, F&& f) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar branches
  const int nfull = (int)((te - ts) / WCH);
  const bool ragged = (te - ts) % WCH != 0;
  const auto Y = gptr((const float*)d.y);
  const int m = d.m;
  // rows 16 bj + r of this lane; only the last block can pass m (m > 16 (MB - 1)):
  // it reads row m - 1 instead and zeroes what it read
  const bool pad = 16 * (MB - 1) + r >= m;
  const __attribute__((address_space(1))) float* Arow[MB];
#pragma unroll
  for (int bj = 0; bj < MB; ++bj) {
    const int row = (bj == MB - 1 && pad) ? m - 1 : 16 * bj + r;
    Arow[bj] = gptr((const float*)d.A + (int64_t)row * d.lda);
  }
  auto load_whole = [&](int c, float (&yv)[WSL], float (&av)[MB][WSL]) __attribute__((always_inline)) {
    const int64_t eb = ts + (int64_t)c * WCH + 4 * g;
    ld_vec_whole<float>(Y, eb, yv);
    ld_vec_whole<float>(Y, eb + 16, yv + 4);
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) {
      ld_vec_whole<float>(Arow[bj], eb, av[bj]);
      ld_vec_whole<float>(Arow[bj], eb + 16, av[bj] + 4);
    }
  };
  // the padded rows are zeroed when a buffer is used, not when it is loaded
  // (a select right after the loads would wait for them and stall the prefetch)
  const bool any_pad = 16 * MB > m;
  auto use = [&](float (&yv)[WSL], float (&av)[MB][WSL], int c) __attribute__((always_inline)) {
    if (any_pad) {
#pragma unroll
      for (int s = 0; s < WSL; ++s) av[MB - 1][s] = pad ? 0.f : av[MB - 1][s];
    }
    f(yv, av, ts + (int64_t)c * WCH, true);
  };
  float y0[WSL], a0[MB][WSL], y1[WSL], a1[MB][WSL];
  int c = w;
  if (c < nfull) load_whole(c, y0, a0);
  // sched_barrier: the next chunk's loads stay ahead of the current chunk's
  // work (left alone, the scheduler sinks them behind it to save registers,
  // which leaves no load in flight while a chunk is being used)
  while (c < nfull) {
    if (c + NWAVE < nfull) load_whole(c + NWAVE, y1, a1);
    __builtin_amdgcn_sched_barrier(0);
    use(y0, a0, c);
    c += NWAVE;
    if (c >= nfull) break;
    if (c + NWAVE < nfull) load_whole(c + NWAVE, y0, a0);
    __builtin_amdgcn_sched_barrier(0);
    use(y1, a1, c);
    c += NWAVE;
  }
  if (ragged && w == nfull % NWAVE) {
    const int64_t e0 = ts + (int64_t)nfull * WCH;
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      const int64_t e = e0 + elem_off(g, s);
      const int64_t ec = e < te ? e : te - 1;
      const float v = Y[ec];
      y0[s] = e < te ? v : 0.f;
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) {
        const float q = Arow[bj][ec];
        a0[bj][s] = (e < te && !(bj == MB - 1 && pad)) ? q : 0.f;
      }
    }
    f(y0, a0, e0, false);
  }
}

// ------------------------------------------------------------------ tile partials

// vals[bj][k]: this lane's sums for row 16 bj + r.  Adds them over the four
// row groups of the wave and then over the waves (fixed order) and publishes
// dst[vidx(j, k)] for rows j < m.  Bit k of kmax: value k is a maximum.
template <int MB, int K, class VI>
__device__ __forceinline__ void rows_to_part(ShW& sh, double (&vals)[MB][K], int m, uint32_t kmax, double* dst,
                                             VI vidx) {
  static_assert(K * 16 * NWAVE <= NWAVE * 256, "per-row values fit the reduction buffer");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int bj = 0; bj < MB; ++bj)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool mx = (kmax >> k) & 1u;
      double v = vals[bj][k];
      double o = __shfl_xor(v, 16, 64);
      v = mx ? fmax(v, o) : v + o;
      o = __shfl_xor(v, 32, 64);
      vals[bj][k] = mx ? fmax(v, o) : v + o;
    }
#pragma unroll
  for (int bj = 0; bj < MB; ++bj) {
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) sh.red.d[(w * K + k) * 16 + r] = vals[bj][k];
    }
    __syncthreads();
    if (tid < K * 16) {
      const int k = tid >> 4, rr = tid & 15, j = 16 * bj + rr;
      const bool mx = (kmax >> k) & 1u;
      double s = sh.red.d[k * 16 + rr];
      for (int ww = 1; ww < NWAVE; ++ww) {
        const double q = sh.red.d[(ww * K + k) * 16 + rr];
        s = mx ? fmax(s, q) : s + q;
      }
      if (j < m) publish(dst + vidx(j, k), s);
    }
    __syncthreads();
  }
}

// Per-lane scalar sums over the workgroup (wave butterflies, then the waves
// in order), published to dst[0..K).
template <int K>
__device__ __forceinline__ void scalars_to_part(ShW& sh, double (&v)[K], double* dst) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh.red.d[w * K + k] = v[k];
  }
  __syncthreads();
  if (tid < K) {
    double s = sh.red.d[tid];
    for (int ww = 1; ww < NWAVE; ++ww) s += sh.red.d[ww * K + tid];
    publish(dst + tid, s);
  }
  __syncthreads();
}

// The float32 J blocks of every wave, added over the waves in float64 (fixed
// order), published as the packed upper triangle.
template <int MB>
__device__ __forceinline__ void jblocks_to_part(ShW& sh, const wf32x4 (&acc)[WN<MB>::NB], int m, double* dstJ) {
  constexpr int NB = WN<MB>::NB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (b0 + u < NB)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh.red.f[((w * 2 + u) * 64 + lane) * 4 + q] = acc[b0 + u][q];
    __syncthreads();
    const int u = tid >> 8, l = (tid >> 2) & 63, q = tid & 3;
    if (b0 + u < NB) {
      double s = (double)sh.red.f[(u * 64 + l) * 4 + q];
      for (int ww = 1; ww < NWAVE; ++ww) s += (double)sh.red.f[((ww * 2 + u) * 64 + l) * 4 + q];
      int bj, bk;
      block_rc<MB>(b0 + u, bj, bk);
      const int j = 16 * bj + 4 * (l >> 4) + q, k = 16 * bk + (l & 15);
      if (j < m && k < m && j <= k) publish(dstJ + pk(j, k, m), s);
    }
    __syncthreads();
  }
}

// The float64 candidate blocks (register q of lane l: candidate i = l / 16 +
// 4 q, row k = 16 bk + l % 16), added over the waves, published at dst[i m + k].
template <int MB>
__device__ __forceinline__ void cblocks_to_part(ShW& sh, const wf64x4 (&acc)[MB], int m, int nc, double* dst) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int bk = 0; bk < MB; ++bk) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sh.red.d[(w * 64 + lane) * 4 + q] = acc[bk][q];
    __syncthreads();
    if (tid < 256) {
      const int l = tid >> 2, q = tid & 3;
      double s = sh.red.d[l * 4 + q];
      for (int ww = 1; ww < NWAVE; ++ww) s += sh.red.d[(ww * 64 + l) * 4 + q];
      const int i = (l >> 4) + 4 * q, k = 16 * bk + (l & 15);
      if (i < nc && k < m) publish(dst + i * m + k, s);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ passes over one tile

// lam = 0 (Alg. 2 start): per row a.clip(y), the free slope sum, the largest
// breakpoint, a.(saturated point), sum |a|, max |a|; non-finite count.
template <int MB>
__device__ __forceinline__ void tile_zero(ShW& sh, const Desc& d, int64_t ts, int64_t te, double* dst) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int m = d.m;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  double acc[MB][6];
#pragma unroll
  for (int bj = 0; bj < MB; ++bj)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[bj][k] = (k == 2) ? -INFINITY : 0.0;
  double bad[1] = {0.0};
  wide_chunks<MB>(d, ts, te, [&](const float (&yv)[WSL], const float (&av)[MB][WSL], int64_t e0, bool whole) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      const double y = (double)yv[s];
      const double x0 = clampd(y, lo, hi);
      const bool fr = (y >= lo) && (y <= hi);
      if (r == 0 && (whole || e0 + elem_off(g, s) < te) && !isfinite(y)) bad[0] += 1.0;
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) {
        const double a = (double)av[bj][s];
        acc[bj][0] = fma(a, x0, acc[bj][0]);
        if (fr) acc[bj][1] = fma(a, a, acc[bj][1]);
        if (a != 0.0) {
          const double bound = (a > 0.0) ? lo : hi;
          acc[bj][2] = fmax(acc[bj][2], breakpoint(y, a, bound));
          acc[bj][3] = fma(a, bound, acc[bj][3]);
        }
        acc[bj][4] += fabs(a);
        acc[bj][5] = fmax(acc[bj][5], fabs(a));
        if (!isfinite(a)) bad[0] += 1.0;
      }
    }
  });
  rows_to_part<MB, 6>(sh, acc, m, (1u << 2) | (1u << 5), dst,
                      [m](int j, int k) { return k < 5 ? k * m + j : 5 * m + 1 + j; });
  scalars_to_part<1>(sh, bad, dst + 5 * m);
}

// Stage 1: for every searching row j its two trials lam_jt alone: a_j.clip(y -
// lam_jt a_j) and the free slope sum (rows not searching carry 0 and are
// ignored by the control).
template <int MB>
__device__ __forceinline__ void tile_stage1(ShW& sh, const Desc& d, int64_t ts, int64_t te, double* dst) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int m = d.m;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  double lt[MB][NT], acc[MB][2 * NT];
#pragma unroll
  for (int bj = 0; bj < MB; ++bj) {
    const int row = 16 * bj + r;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double v = row < m ? sh.pay[NT * row + t] : 0.0;
      lt[bj][t] = (v == v) ? v : 0.0;
      acc[bj][2 * t] = 0.0;
      acc[bj][2 * t + 1] = 0.0;
    }
  }
  wide_chunks<MB>(d, ts, te, [&](const float (&yv)[WSL], const float (&av)[MB][WSL], int64_t, bool) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      const double yq = (double)yv[s];
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) {
        const double a = (double)av[bj][s];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const double z = fma(-lt[bj][t], a, yq);
          acc[bj][2 * t] = fma(a, clampd(z, lo, hi), acc[bj][2 * t]);
          if (z >= lo && z <= hi) acc[bj][2 * t + 1] = fma(a, a, acc[bj][2 * t + 1]);
        }
      }
    }
  });
  rows_to_part<MB, 2 * NT>(sh, acc, m, 0u, dst, [](int j, int k) { return 2 * NT * j + k; });
}

// Stage-1 check: C[i][k] = a_k . clip(y - lam_i a_{c_i}) for the candidates
// c_i of this pass (float64 matrix cores: the A operand is the candidates'
// clipped points, the B operand the rows).
template <int MB>
__device__ __forceinline__ void tile_check(ShW& sh, const Desc& d, int64_t ts, int64_t te, double* dst) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int m = d.m, nc = sh.aux;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  const int crow = r < nc ? (int)sh.pay[WCAND + r] : -1;
  const double clam = r < nc ? sh.pay[r] : 0.0;
  const auto Ac = gptr((const float*)d.A + (int64_t)(crow < 0 ? 0 : crow) * d.lda);
  wf64x4 acc[MB];
#pragma unroll
  for (int bk = 0; bk < MB; ++bk) acc[bk] = wf64x4{0.0, 0.0, 0.0, 0.0};
  wide_chunks<MB>(d, ts, te, [&](const float (&yv)[WSL], const float (&av)[MB][WSL], int64_t e0, bool whole) __attribute__((always_inline)) {
    const int64_t eb = e0 + 4 * g;
    float ac[WSL];
    if (whole) {
      if (crow >= 0) {
        ld_vec_whole<float>(Ac, eb, ac);
        ld_vec_whole<float>(Ac, eb + 16, ac + 4);
      } else {
#pragma unroll
        for (int s = 0; s < WSL; ++s) ac[s] = 0.f;
      }
    } else {
#pragma unroll
      for (int s = 0; s < WSL; ++s) {
        const int64_t e = e0 + elem_off(g, s);
        const int64_t ec = e < te ? e : te - 1;
        float v = 0.f;
        if (crow >= 0) v = Ac[ec];
        ac[s] = e < te ? v : 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      // past the tile end the rows are zero, so whatever xc is adds nothing
      const double xc = crow >= 0 ? clampd(fma(-clam, (double)ac[s], (double)yv[s]), lo, hi) : 0.0;
#pragma unroll
      for (int bk = 0; bk < MB; ++bk)
        acc[bk] = __builtin_amdgcn_mfma_f64_16x16x4f64(xc, (double)av[bk][s], acc[bk], 0, 0, 0);
    }
  });
  cblocks_to_part<MB>(sh, acc, m, nc, dst);
}

// Newton pass at the trial lam: h_j + b_j + kappa lam_j = a_j.x(lam) (float64)
// and J = A D A^T (float32 matrix cores on the free-masked tile).
template <int MB>
__device__ __forceinline__ void tile_newton(ShW& sh, const Desc& d, int64_t ts, int64_t te, double* dst) {
  constexpr int NB = WN<MB>::NB;
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int m = d.m;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  double lamr[MB], hacc[MB][1];
#pragma unroll
  for (int bj = 0; bj < MB; ++bj) {
    const int row = 16 * bj + r;
    lamr[bj] = row < m ? sh.pay[row] : 0.0;
    hacc[bj][0] = 0.0;
  }
  wf32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = wf32x4{0.f, 0.f, 0.f, 0.f};
  wide_chunks<MB>(d, ts, te, [&](const float (&yv)[WSL], const float (&av)[MB][WSL], int64_t, bool) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      double p = 0.0;
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) p = fma(lamr[bj], (double)av[bj][s], p);
      p = row_sum16(p);
      const double z = (double)yv[s] - p;
      const double x = clampd(z, lo, hi);
      const bool fr = (z >= lo) && (z <= hi);
      float fa[MB];
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) {
        hacc[bj][0] = fma((double)av[bj][s], x, hacc[bj][0]);
        fa[bj] = fr ? av[bj][s] : 0.f;
      }
      int b = 0;
#pragma unroll
      for (int bj = 0; bj < MB; ++bj)
#pragma unroll
        for (int bk = bj; bk < MB; ++bk) {
          acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[bj], fa[bk], acc[b], 0, 0, 0);
          ++b;
        }
    }
  });
  rows_to_part<MB, 1>(sh, hacc, m, 0u, dst, [](int j, int) { return j; });
  jblocks_to_part<MB>(sh, acc, m, dst + m);
}

// Final pass: x = clip(y - A^T lam) stored, a.x per row of x as stored, the
// free count, |x - y|^2, free-mask words (one per chunk).
template <int MB>
__device__ __forceinline__ void tile_final(ShW& sh, const Desc& d, int64_t ts, int64_t te, double* dst) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int m = d.m;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  float* X = (float*)d.x;
  double lamr[MB], acc[MB][1];
#pragma unroll
  for (int bj = 0; bj < MB; ++bj) {
    const int row = 16 * bj + r;
    lamr[bj] = row < m ? sh.pay[row] : 0.0;
    acc[bj][0] = 0.0;
  }
  double sc[4] = {0.0, 0.0, 0.0, 0.0};   // free count, (pgd terms unused), |x - y|^2
  wide_chunks<MB>(d, ts, te, [&](const float (&yv)[WSL], const float (&av)[MB][WSL], int64_t e0, bool whole) __attribute__((always_inline)) {
    float xo[WSL];
    uint32_t bits = 0;
#pragma unroll
    for (int s = 0; s < WSL; ++s) {
      double p = 0.0;
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) p = fma(lamr[bj], (double)av[bj][s], p);
      p = row_sum16(p);
      const double z = (double)yv[s] - p;
      xo[s] = (float)clampd(z, lo, hi);
      const bool valid = whole || e0 + elem_off(g, s) < te;
      if (valid && z >= lo && z <= hi) bits |= 1u << s;
      const double xr = (double)xo[s];
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) acc[bj][0] = fma((double)av[bj][s], xr, acc[bj][0]);
      if (r == 0 && valid) {
        const double dy = xr - (double)yv[s];
        sc[3] = fma(dy, dy, sc[3]);
      }
    }
    if (r == 0) sc[0] += (double)__builtin_popcount(bits);
    if (whole) {
      if (r < 2) {
        const wf32x4 v = (r == 0) ? wf32x4{xo[0], xo[1], xo[2], xo[3]} : wf32x4{xo[4], xo[5], xo[6], xo[7]};
        *reinterpret_cast<__attribute__((address_space(1))) wf32x4*>(gptr_w(X) + e0 + 4 * g + 16 * r) = v;
      }
    } else if (r == 0) {
#pragma unroll
      for (int s = 0; s < WSL; ++s) {
        const int64_t e = e0 + elem_off(g, s);
        if (e < te) gptr_w(X)[e] = xo[s];
      }
    }
    if (d.free_mask) {
      // bit elem_off(g, s) of the chunk's word: the group's low nibble at 4 g, high nibble at 16 + 4 g
      uint32_t word = 0;
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        const uint32_t b = (uint32_t)__shfl((int)bits, 16 * gg, 64);
        word |= ((b & 0xFu) << (4 * gg)) | ((b >> 4) << (16 + 4 * gg));
      }
      if (lane == 0) d.free_mask[e0 >> 5] = word;
    }
  });
  rows_to_part<MB, 1>(sh, acc, m, 0u, dst, [](int j, int) { return j; });
  scalars_to_part<4>(sh, sc, dst + m);
}

// ------------------------------------------------------------------ pass values

__device__ __forceinline__ int wide_nv(int ph, int m, int aux) {
  switch (ph) {
    case PH_ZERO: return 6 * m + 1;
    case PH_STAGE1: return 2 * NT * m;
    case PH_CHECK: return aux * m;
    case PH_NEWTON: return m + m * (m + 1) / 2;
    default: return m + 4;
  }
}

__device__ __forceinline__ bool wide_is_max(int ph, int v, int m) {
  return ph == PH_ZERO && ((v >= 2 * m && v < 3 * m) || v >= 5 * m + 1);
}

// ------------------------------------------------------------------ Newton control (workgroup 0, all threads)

// Continuous NCP (or the paper's), as in the small kernel: c = J_jj + kappa.
__device__ __forceinline__ void wide_ncp(int mode, bool eqj, double h, double lam, double c, double& phi, int& act) {
  if (eqj) {
    act = 1;
    phi = h;
  } else if (mode == PGDTO_NCP_PAPER) {
    act = h > 0.0;
    phi = act ? h : (h < 0.0 ? -lam : 0.0);
  } else {
    act = h + c * lam > 0.0;
    phi = act ? h : -c * lam;
  }
}

// Semismooth Newton direction (Appendix A.2): rows outside the active set
// release their multiplier, the active rows solve
// (J + kappa I)_SS Delta_S = h_S - (J + kappa I)_SN Delta_N.
// The active block is factored as L D L^T by the whole workgroup: thread t
// keeps row a = t / 8, columns b = t % 8 + 8 q (q < 8) of the block in
// registers; step j publishes column j through LDS, every thread updates
// its entries with it; one barrier per step.  The factor L (packed lower
// triangle) then overwrites the Jacobian sums in sh.tot, and one wave
// solves the two triangular systems with the unknowns in lanes.
// Reads sh.lam, sh.h, sh.act, sh.phi; writes sh.delta.
// Row sums of the control by 8 threads per row (thread t: row t / 8, terms
// k = t % 8, t % 8 + 8, ...), added over the 8 threads with a fixed xor
// pattern, so every thread of the row holds the same bits.
__device__ __forceinline__ double row8_sum(double part) {
  part += __shfl_xor(part, 1, 64);
  part += __shfl_xor(part, 2, 64);
  part += __shfl_xor(part, 4, 64);
  return part;
}

__device__ void wide_direction(ShW& sh, double* J, int m) {
  const int tid = threadIdx.x;
  const double kappa = sh.kappa;
  const int mode = sh.ncp;
  if (tid < m) sh.delta[tid] = sh.act[tid] ? 0.0 : (mode == PGDTO_NCP_PAPER ? sh.phi[tid] : -sh.lam[tid]);
  if (tid < 64) {
    // active rows in index order: a ballot and a prefix count
    const bool on = tid < m && sh.act[tid];
    const uint64_t msk = __ballot(on);
    if (on) sh.sidx[__popcll(msk & ((1ull << tid) - 1ull))] = tid;
    if (tid == 0) sh.np = __popcll(msk);
  }
  __syncthreads();
  const int p = sh.np;
  {
    // rhs_r = h_j - sum over inactive k of (J + kappa I)_jk delta_k, j = sidx[r]
    const int r = tid >> 3, c = tid & 7;
    double part = 0.0;
    if (r < p) {
      const int j = sh.sidx[r];
      for (int k = c; k < m; k += 8)
        if (!sh.act[k]) part = fma(J[pks(j, k, m)] + (j == k ? kappa : 0.0), sh.delta[k], part);
    }
    part = row8_sum(part);
    if (r < p && c == 0) sh.rhs[r] = sh.h[sh.sidx[r]] - part;
  }
  const int a = tid >> 3, c0 = tid & 7;
  double K[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int b = c0 + 8 * q;
    K[q] = (a < p && b <= a) ? J[pk(sh.sidx[b], sh.sidx[a], m)] + (a == b ? kappa : 0.0) : 0.0;
  }
  __syncthreads();   // every read of J is done: the factor may overwrite it
  for (int j = 0; j < p; ++j) {
    const int qj = j >> 3;
    if (c0 == (j & 7) && a >= j && a < p) {
      double kv = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) kv = (q == qj) ? K[q] : kv;
      sh.colbuf[j & 1][a] = kv;
    }
    __syncthreads();
    double Dj = sh.colbuf[j & 1][j];
    if (!(Dj > 0.0)) Dj = fmax(kappa, 1e-300);    // a pivot lost to rounding (J is PSD)
    const double inv = 1.0 / Dj;
    if (a > j && a < p) {
      const double ca = sh.colbuf[j & 1][a];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = c0 + 8 * q;
        if (b > j && b <= a) K[q] = fma(-ca, sh.colbuf[j & 1][b] * inv, K[q]);
      }
      if (c0 == 0) J[(a * (a + 1)) / 2 + j] = ca * inv;
    }
    if (tid == 0) sh.dv[j] = Dj;
  }
  __syncthreads();
  if (tid < 64) {
    const int ln = tid;
    double u = ln < p ? sh.rhs[ln] : 0.0;
    for (int b = 0; b < p; ++b) {           // L u = rhs (unit lower)
      const double ub = lane_value(u, b);
      if (ln > b && ln < p) u = fma(-J[(ln * (ln + 1)) / 2 + b], ub, u);
    }
    double v = ln < p ? u / sh.dv[ln] : 0.0;
    for (int b = p - 1; b >= 0; --b) {      // L^T w = D^-1 u
      const double wb = lane_value(v, b);
      if (ln < b) v = fma(-J[(b * (b + 1)) / 2 + ln], wb, v);
    }
    if (ln < p) sh.delta[sh.sidx[ln]] = v;
  }
  __syncthreads();
  if (tid == 0) sh.tmark[1] = clk();
}

// Accept (lam, h, J) as the iterate: stop (returns PH_FINAL, payload = the
// multipliers) or take the Newton step (PH_NEWTON, payload = the first trial).
// J (packed, in LDS) is consumed.
__device__ int wide_accept(ShW& sh, const double* lam_in, const double* h_in, double* J, int m) {
  const int tid = threadIdx.x;
  const double kappa = sh.kappa;
  if (tid < m) {
    sh.lam[tid] = lam_in[tid];
    sh.h[tid] = h_in[tid];
  }
  __syncthreads();
  if (tid < m) {
    const int j = tid;
    const bool eqj = (sh.eq >> j) & 1ull;
    const double c = J[pk(j, j, m)] + kappa;
    sh.diagc[j] = c;
    const double h = sh.h[j], lam = sh.lam[j];
    sh.rowv[j] = ((eqj || lam > 0.0) ? fabs(h) : fmax(h, 0.0)) / sh.S.scale[j];
    double phi;
    int act;
    wide_ncp(sh.ncp, eqj, h, lam, c, phi, act);
    sh.phi[j] = phi;
    sh.act[j] = act;
  }
  __syncthreads();
  if (tid < 64) {
    const double res = wave_max(tid < m ? sh.rowv[tid] : 0.0);
    const double ph = tid < m ? sh.phi[tid] : 0.0;
    const double p2 = wave_sum(ph * ph);
    if (tid == 0) {
      sh.res_inf = res;
      sh.p2 = p2;
    }
  }
  wide_direction(sh, J, m);
  const bool stop = sh.res_inf <= sh.tol_n || sh.it >= sh.max_newton;
  if (stop) {
    if (tid < m) {
      sh.lamf[tid] = sh.lam[tid];
      sh.lerr[tid] = 2.0 * fabs(sh.delta[tid]);     // the step at the returned multipliers, doubled
      sh.lslope[tid] = sh.diagc[tid];
      sh.pay[tid] = sh.lam[tid];
    }
    if (tid == 0) sh.outcome = sh.res_inf <= sh.tol_n ? PGDTO_CONVERGED : PGDTO_MAXITER;
    __syncthreads();
    return PH_FINAL;
  }
  if (tid < m) {
    const bool eqj = (sh.eq >> tid) & 1ull;
    const double t = sh.lam[tid] + sh.delta[tid];
    sh.pay[tid] = eqj ? t : fmax(t, 0.0);
  }
  if (tid == 0) {
    sh.phi2 = sh.p2;
    sh.M0 = 0.5 * sh.p2;
    sh.gamma = 1.0;
    sh.ls = 0;
    sh.have_best = 0;
    sh.it += 1;
  }
  __syncthreads();
  return PH_NEWTON;
}

// Line-search decision after evaluating the trial (tr = sh.pay, ht = sh.htr,
// J = the trial's sums): Armijo (c1) and curvature (c2) conditions, halving
// gamma from 1 (Appendix A.2); the first Armijo trial is kept as a fallback.
__device__ int wide_after_trial(ShW& sh, const WSync& W, double* J, int m) {
  enum { HALVE = 0, ACCEPT_TRIAL = 1, ACCEPT_BEST = 2, KEEP = 4 };
  const int tid = threadIdx.x;
  const double kappa = sh.kappa;
  {
    // row j of J_Phi delta (8 threads per row), then Phi_j times it
    const int j = tid >> 3, cc = tid & 7;
    double phi = 0.0, part = 0.0, c = 0.0;
    int act = 0;
    if (j < m) {
      const bool eqj = (sh.eq >> j) & 1ull;
      c = J[pk(j, j, m)] + kappa;
      wide_ncp(sh.ncp, eqj, sh.htr[j], sh.pay[j], c, phi, act);
      if (act)
        for (int k = cc; k < m; k += 8) part = fma(J[pks(j, k, m)] + (j == k ? kappa : 0.0), sh.delta[k], part);
    }
    part = row8_sum(part);
    if (j < m && cc == 0) {
      const double row = act ? part : ((sh.ncp == PGDTO_NCP_PAPER) ? sh.delta[j] : c * sh.delta[j]);
      sh.phi[j] = phi;
      sh.rowv[j] = phi * row;
    }
  }
  __syncthreads();
  if (tid < 64) {
    const double ph = tid < m ? sh.phi[tid] : 0.0;
    const double p2 = wave_sum(ph * ph);
    const double gd = wave_sum(tid < m ? sh.rowv[tid] : 0.0);
    if (tid == 0) {
      const bool armijo = 0.5 * p2 <= sh.M0 - sh.c1 * sh.gamma * sh.phi2;
      const bool curv = gd <= sh.c2 * sh.phi2;
      const int hb = sh.have_best, ls = sh.ls + 1;
      sh.ls = ls;
      int dec;
      if (armijo && curv) dec = ACCEPT_TRIAL;
      else if (ls >= sh.max_ls) dec = hb ? ACCEPT_BEST : ACCEPT_TRIAL;
      else dec = HALVE;
      if (armijo && !hb) dec |= KEEP;
      sh.decision = dec;
    }
  }
  __syncthreads();
  const int dec = sh.decision;
  if (dec & KEEP) {
    const int nj = m * (m + 1) / 2;
    for (int i = tid; i < nj; i += BLOCK) publish(W.best + i, J[i]);
    if (tid < m) {
      sh.blam[tid] = sh.pay[tid];
      sh.bh[tid] = sh.htr[tid];
    }
    if (tid == 0) sh.have_best = 1;
    wait_own_stores();
    __syncthreads();
  }
  if ((dec & 3) == ACCEPT_TRIAL) return wide_accept(sh, sh.pay, sh.htr, J, m);
  if ((dec & 3) == ACCEPT_BEST) {
    const int nj = m * (m + 1) / 2;
    for (int i = tid; i < nj; i += BLOCK) J[i] = fetch_published(W.best + i);
    __syncthreads();
    return wide_accept(sh, sh.blam, sh.bh, J, m);
  }
  const double gnew = 0.5 * sh.gamma;
  if (tid < m) {
    const bool eqj = (sh.eq >> tid) & 1ull;
    const double t = sh.lam[tid] + gnew * sh.delta[tid];
    sh.pay[tid] = eqj ? t : fmax(t, 0.0);
  }
  __syncthreads();
  if (tid == 0) sh.gamma = gnew;
  return PH_NEWTON;
}

// Candidates of the next check pass: rows with a positive Stage-1
// multiplier, in index order from sh.cnext, at most WCAND.  Returns their count.
__device__ int wide_next_candidates(ShW& sh, int m) {
  int nc = 0, j = sh.cnext;
  for (; j < m && nc < WCAND; ++j) {
    if (sh.lam1[j] > 0.0) {
      sh.pay[nc] = sh.lam1[j];
      sh.pay[WCAND + nc] = (double)j;
      ++nc;
    }
  }
  sh.cnext = j;
  sh.aux = nc;
  return nc;
}

// Thread 0: after Stage 1 (or without it), the check of the candidates, or
// Newton from the Stage-1 multipliers when there is none.
__device__ int wide_after_stage1(ShW& sh, int m) {
  for (int j = 0; j < m; ++j) sh.lam1[j] = sh.S.lam[j];
  sh.cnext = 0;
  if (wide_next_candidates(sh, m) > 0) return PH_CHECK;
  sh.path = 3;
  for (int j = 0; j < m; ++j) sh.pay[j] = sh.lam1[j];
  sh.init = 1;
  return PH_NEWTON;
}

// Result of the solve (workgroup 0), from the totals of the final pass.
__device__ void wide_result(ShW& sh, const Desc& d, int m) {
  const int tid = threadIdx.x;
  const double* t = sh.tot;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  const double kappa = sh.kappa;
  pgdto_result* R = (pgdto_result*)d.result;
  if (tid < m) {
    const int j = tid;
    const bool eqj = (sh.eq >> j) & 1ull;
    const double lamj = sh.lamf[j];
    R->lambda[j] = lamj;
    R->resid[j] = t[j] - sh.bs[j];
    R->slack[j] = kappa * lamj;
    int o = (eqj || lamj > 0.0) ? PGDTO_CONVERGED : PGDTO_INACTIVE;
    if (sh.S.ssat[j] - sh.bs[j] > 0.0) o = PGDTO_INFEASIBLE;
    if (eqj && sh.bs[j] - (sh.S.ssat[j] + sh.asum[j] * (hi - lo)) > 0.0) o = PGDTO_INFEASIBLE;
    if (sh.outcome == PGDTO_MAXITER || sh.outcome == PGDTO_NONFINITE) o = sh.outcome;
    R->row_outcome[j] = o;
    const double le = sh.nonfinite ? INFINITY : lam_error(lamj, sh.lerr[j], sh.S.scale[j], sh.lslope[j]);
    R->lambda_err[j] = le;
    const double h = t[j] - sh.bs[j] - kappa * lamj;
    sh.rowv[j] = ((eqj || lamj != 0.0) ? fabs(h) : fmax(h, 0.0)) / sh.S.scale[j];
    sh.rhs[j] = le;
    sh.act[j] = o;
  }
  __syncthreads();
  if (tid == 0) {
    int worst = sh.outcome;
    double rmax = 0.0, xerr = 0.0, wmax = 0.0;
    int np = 0;
    for (int j = 0; j < m; ++j) {
      if (sh.act[j] == PGDTO_INFEASIBLE && severity(PGDTO_INFEASIBLE) > severity(worst)) worst = PGDTO_INFEASIBLE;
      rmax = fmax(rmax, sh.rowv[j]);
      xerr += sh.amax[j] * sh.rhs[j];
      wmax = fmax(wmax, sh.S.width[j]);
      np = max(np, sh.S.npass[j]);
    }
    R->outcome = worst;
    R->error = 0;
    R->path = sh.path;
    R->passes = sh.passes + 1;
    R->iters_search = np;
    R->iters_newton = sh.it;
    R->iters_ls = sh.ls_total;
    R->m = m;
    R->n_free = (int64_t)t[m];
    R->res_inf = rmax;
    R->n_compact = -1;
    R->passes_compacted = 0;
    R->dist2 = t[m + 3];
    R->x_err = xerr + half_ulp(fmax(fabs(lo), fabs(hi)), true);
    R->lambda_width = wmax;
    R->kappa = kappa;
  }
  __syncthreads();
}

// The control after a pass (workgroup 0, all threads): reads sh.tot, sets the
// next command (sh.ph, sh.aux, sh.pay).
__device__ void wide_control(ShW& sh, const Desc& d, const WSync& W, int ph) {
  const int tid = threadIdx.x;
  const int m = d.m;
  const double* t = sh.tot;
  const double lo = __builtin_canonicalize(d.lo), hi = __builtin_canonicalize(d.hi);
  if (ph == PH_ZERO) {
    if (tid == 0 && d.auto_tau > 0.0) sh.kappa = auto_kappa(d.auto_tau, &t[2 * m], 1, m);
    __syncthreads();
    const double kappa = sh.kappa;
    if (tid < m) {
      const int j = tid;
      double scale = t[4 * m + j] * fmax(fabs(lo), fabs(hi));
      if (!(scale > 0.0)) scale = 1.0;
      sh.S.scale[j] = scale;
      sh.amax[j] = t[5 * m + 1 + j];
      sh.asum[j] = t[4 * m + j];
      sh.S.slope[j] = t[m + j] + kappa;
      sh.h0[j] = t[j] - sh.bs[j];
      sh.S.ssat[j] = t[3 * m + j];
      if (d.stage1 && !d.eq_mask && !d.warm && t[5 * m] == 0.0) {
        search_init(sh.S, j, t[j] - sh.bs[j], t[m + j] + kappa, t[2 * m + j], t[3 * m + j], sh.bs[j], kappa,
                    scale, sh.search, false);
      } else {
        sh.S.state[j] = SEG_DONE;
        sh.S.lam[j] = 0.0;
        sh.S.npass[j] = 0;
      }
    }
    __syncthreads();
    if (tid == 0) {
      sh.passes += 1;
      bool any_pos = false;
      for (int j = 0; j < m; ++j) any_pos |= ((sh.eq >> j) & 1ull) ? (sh.h0[j] != 0.0) : (sh.h0[j] > 0.0);
      int next;
      if (t[5 * m] > 0.0) {
        sh.nonfinite = 1;
        sh.outcome = PGDTO_NONFINITE;
        next = PH_FINAL;
      } else if (!any_pos) {
        sh.outcome = PGDTO_INACTIVE;
        sh.path = 0;
        next = PH_FINAL;
      } else if (!d.stage1 || d.eq_mask || d.warm) {
        sh.path = 3;
        for (int j = 0; j < m; ++j) sh.pay[j] = d.warm ? d.lam0[j] : 0.0;
        sh.init = 1;
        next = PH_NEWTON;
      } else {
        int any = 0;
        for (int j = 0; j < m; ++j) any |= (sh.S.state[j] == SEG_SEARCH);
        next = any ? PH_STAGE1 : wide_after_stage1(sh, m);
      }
      if (next == PH_FINAL)
        for (int j = 0; j < m; ++j) sh.pay[j] = 0.0;
      sh.ph = next;
    }
  } else if (ph == PH_STAGE1) {
    if (tid < m && sh.S.state[tid] == SEG_SEARCH) {
      const int j = tid;
      search_update(sh.S, j, t[2 * NT * j], t[2 * NT * j + 2], t[2 * NT * j + 1], t[2 * NT * j + 3], sh.bs[j],
                    sh.kappa, sh.tol_n, sh.tol_b, sh.max_search, sh.search, false);
    }
    __syncthreads();
    if (tid == 0) {
      sh.passes += 1;
      sh.s1passes += 1;
      int any = 0;
      for (int j = 0; j < m; ++j) any |= (sh.S.state[j] == SEG_SEARCH);
      sh.ph = any ? PH_STAGE1 : wide_after_stage1(sh, m);
    }
  } else if (ph == PH_CHECK) {
    const int nc = sh.aux;
    if (tid < nc) {
      const int c = (int)sh.pay[WCAND + tid];
      const double lc = sh.pay[tid];
      bool ok = true;
      for (int k = 0; k < m && ok; ++k) {
        const double hk = t[tid * m + k] - sh.bs[k] - (k == c ? sh.kappa * lc : 0.0);
        if (hk > sh.tol_n * sh.S.scale[k]) ok = false;
      }
      sh.rowv[tid] = ok ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      sh.passes += 1;
      int found = -1;
      for (int i = 0; i < nc && found < 0; ++i)
        if (sh.rowv[i] != 0.0) found = (int)sh.pay[WCAND + i];
      if (found >= 0) {
        for (int j = 0; j < m; ++j) {
          sh.lamf[j] = (j == found) ? sh.lam1[j] : 0.0;
          sh.lerr[j] = (j == found) ? sh.S.err[j] : 0.0;
          sh.lslope[j] = sh.S.slope[j];
          sh.pay[j] = sh.lamf[j];
        }
        sh.path = 2;
        sh.outcome = PGDTO_CONVERGED;
        sh.ph = PH_FINAL;
      } else if (wide_next_candidates(sh, m) > 0) {
        sh.ph = PH_CHECK;
      } else {
        sh.path = 3;
        for (int j = 0; j < m; ++j) sh.pay[j] = sh.lam1[j];
        sh.init = 1;
        sh.ph = PH_NEWTON;
      }
    }
  } else if (ph == PH_NEWTON) {
    const double kappa = sh.kappa;
    if (tid < m) sh.htr[tid] = t[tid] - sh.bs[tid] - kappa * sh.pay[tid];
    if (tid == 0) {
      sh.passes += 1;
      sh.ls_total += 1;
    }
    __syncthreads();
    double* J = sh.tot + m;
    int next;
    if (sh.init) {
      __syncthreads();
      if (tid == 0) sh.init = 0;
      next = wide_accept(sh, sh.pay, sh.htr, J, m);
    } else {
      next = wide_after_trial(sh, W, J, m);
    }
    if (tid == 0) sh.ph = next;
  } else {  // PH_FINAL
    wide_result(sh, d, m);
    if (tid == 0) sh.ph = PH_DONE;
  }
  __syncthreads();
  if (sh.ph == PH_STAGE1 && tid < m) {
#pragma unroll
    for (int t = 0; t < NT; ++t) sh.pay[NT * tid + t] = (sh.S.state[tid] == SEG_SEARCH) ? sh.S.trial[tid][t] : NAN;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ grid synchronisation

// Barrier A: every workgroup raises its flag; workgroup 0 waits for all of
// them and raises the go word on every replica.  Bounded waits: on expiry the
// error line records the launch and every workgroup leaves.
__device__ __forceinline__ bool wide_barrier(ShW& sh, const Desc& d, const WSync& W, uint64_t e) {
  const int tid = threadIdx.x, G = wg_num(d), wid = wg_id(d);
  if (tid == 0) {
    sh.abort_flag = 0;
    __hip_atomic_store(&W.flags[(size_t)wid * FLAG_STRIDE], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (wid == 0) {
    bool ok = true;
    for (int w = tid; w < G && ok; w += BLOCK) {
      uint32_t spins = 0;
      while (__hip_atomic_load(&W.flags[(size_t)w * FLAG_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < e) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT) { ok = false; break; }
      }
    }
    if (!ok) atomicOr(&sh.abort_flag, 1);
    __syncthreads();
    if (sh.abort_flag) {
      if (tid == 0) __hip_atomic_store(W.err, d.epoch0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    return true;
  }
  return true;
}

// A worker's wait for the go word of epoch e on its replica.
__device__ __forceinline__ bool wide_wait_go(ShW& sh, const Desc& d, const WSync& W, uint64_t e) {
  const int wid = wg_id(d);
  uint64_t* my = W.rep + (size_t)(wid % WNREP) * WREP;
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    bool ok = true;
    while (__hip_atomic_load(my, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < e) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT || __hip_atomic_load(W.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == d.epoch0) {
        ok = false;
        break;
      }
    }
    if (!ok) {
      __hip_atomic_store(W.err, d.epoch0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh.abort_flag = 1;
    }
  }
  __syncthreads();
  return !sh.abort_flag;
}

__device__ __forceinline__ void wide_raise_go(const WSync& W, uint64_t e) {
  if (threadIdx.x < WNREP)
    __hip_atomic_store(W.rep + (size_t)threadIdx.x * WREP, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// End of a pass: barrier A (tile partials complete), every workgroup sums a
// slice of the values over all tiles, barrier B with workgroup 0's control
// in it, which publishes the next command with the go word.
__device__ bool wide_sync(ShW& sh, const Desc& d, const WSync& W, int pass, int ph, int nv) {
  const int tid = threadIdx.x, lane = tid & 63, G = wg_num(d), wid = wg_id(d);
  const uint64_t e1 = d.epoch0 + 2 * (uint64_t)pass + 1, e2 = e1 + 1;
  wait_own_stores();
  __syncthreads();
  if (!wide_barrier(sh, d, W, e1)) return false;
  trace_put(d, pass, 2, clk());
  if (wid == 0) wide_raise_go(W, e1);
  else if (!wide_wait_go(sh, d, W, e1)) return false;
  // the partials of every tile are in memory
  const int m = d.m;
  const int per = (nv + G - 1) / G;
  const int v0 = wid * per, v1 = min(nv, v0 + per);
  for (int v = v0 + (tid >> 6); v < v1; v += NWAVE) {
    const bool mx = wide_is_max(ph, v, m);
    double s = mx ? -INFINITY : 0.0;
    for (int t = lane; t < d.ntiles; t += 64) {
      const double q = fetch_published(W.part + (size_t)t * WV_PAD + v);
      s = mx ? fmax(s, q) : s + q;
    }
    s = mx ? wave_max(s) : wave_sum(s);
    if (lane == 0) publish(W.tot + v, s);
  }
  wait_own_stores();
  __syncthreads();
  if (!wide_barrier(sh, d, W, e2)) return false;
  trace_put(d, pass, 3, clk());
  if (wid == 0) {
    for (int i = tid; i < nv; i += BLOCK) sh.tot[i] = fetch_published(W.tot + i);
    __syncthreads();
    if (tid == 0) { sh.tmark[0] = clk(); sh.tmark[1] = 0; }
    wide_control(sh, d, W, ph);
    trace_put(d, pass, 4, clk());
    trace_put(d, pass, 6, sh.tmark[0]);
    trace_put(d, pass, 7, sh.tmark[1]);
    // the command on every replica (the payload words the next pass reads),
    // then the go word
    const int nph = sh.ph;
    const int npay = nph == PH_STAGE1 ? NT * m : nph == PH_CHECK ? 2 * WCAND
                     : (nph == PH_NEWTON || nph == PH_FINAL) ? m : 0;
    const int NW = REP_PAY + npay;
    for (int i = tid; i < WNREP * NW; i += BLOCK) {
      const int rp = i / NW, k = i - rp * NW;
      uint64_t v;
      if (k == 0) continue;
      else if (k == REP_PH) v = (uint64_t)(uint32_t)sh.ph;
      else if (k == REP_AUX) v = (uint64_t)(uint32_t)sh.aux;
      else if (k < REP_PAY) v = 0;
      else v = __builtin_bit_cast(uint64_t, sh.pay[k - REP_PAY]);
      __hip_atomic_store(W.rep + (size_t)rp * WREP + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    wait_own_stores();
    __syncthreads();
    wide_raise_go(W, e2);
    trace_put(d, pass, 5, clk());
    return true;
  }
  if (!wide_wait_go(sh, d, W, e2)) return false;
  const uint64_t* my = W.rep + (size_t)(wid % WNREP) * WREP;
  if (tid == 0) {
    sh.ph = (int32_t)__hip_atomic_load(my + REP_PH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh.aux = (int32_t)__hip_atomic_load(my + REP_AUX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid < 2 * WM)
    sh.pay[tid] = __builtin_bit_cast(double, __hip_atomic_load(my + REP_PAY + tid, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT));
  __syncthreads();
  return true;
}

// ------------------------------------------------------------------ the solver
// Per-pass trace records (contexts created with PGDTO_TRACE): [0] phase << 56
// | start, [1] tiles done, [2] barrier A complete (every partial published),
// [3] barrier B complete (every slice summed), [4] control done, [5] go
// raised, [6] totals in LDS (control starts), [7] last Newton direction solved.

template <int MB>
__device__ void solve_wide(ShW& sh, const Desc& d) {
  const int tid = threadIdx.x;
  const int G = wg_num(d), wid = wg_id(d);
  const int m = d.m;
  const WSync W = wide_words(d);
  if (tid == 0) {
    sh.ph = PH_ZERO;
    sh.aux = 0;
    sh.abort_flag = 0;
    sh.eq = d.eq_mask;
    sh.kappa = d.kappa;
    sh.tol_n = d.tol_n;
    sh.tol_b = d.tol_b;
    sh.c1 = d.c1;
    sh.c2 = d.c2;
    sh.max_newton = d.max_newton;
    sh.max_ls = d.max_ls;
    sh.max_search = d.max_search;
    sh.ncp = d.ncp;
    sh.search = d.search;
    sh.have_best = 0; sh.ls = 0; sh.it = 0; sh.init = 0; sh.passes = 0; sh.path = 0;
    sh.outcome = PGDTO_INACTIVE; sh.nonfinite = 0; sh.s1passes = 0; sh.ls_total = 0; sh.cnext = 0;
    sh.res_inf = 0.0; sh.gamma = 1.0; sh.phi2 = 0.0; sh.M0 = 0.0; sh.p2 = 0.0;
  }
  if (tid < WM) {
    const int j = tid;
    sh.bs[j] = j < m ? d.b[j] : 0.0;
    sh.lamf[j] = 0.0; sh.lerr[j] = 0.0; sh.lslope[j] = 0.0; sh.amax[j] = 0.0; sh.asum[j] = 0.0;
    sh.lam1[j] = 0.0; sh.h0[j] = 0.0;
    sh.S.state[j] = SEG_DONE; sh.S.lam[j] = 0.0; sh.S.npass[j] = 0; sh.S.width[j] = 0.0;
    sh.S.outcome[j] = PGDTO_INACTIVE; sh.S.scale[j] = 1.0; sh.S.ssat[j] = 0.0; sh.S.err[j] = 0.0;
    sh.S.slope[j] = 0.0;
  }
  __syncthreads();
  for (int pass = 0;; ++pass) {
    const int ph = sh.ph;
    if (ph == PH_DONE) break;
    const int nv = wide_nv(ph, m, sh.aux);
    const uint64_t t_pass0 = clk();
    trace_put(d, pass, 0, ((uint64_t)ph << 56) | (t_pass0 & 0x00ffffffffffffffull));
    for (int tile = wid; tile < d.ntiles; tile += G) {
      const int64_t ts = (int64_t)tile * d.tile_elems;
      const int64_t te = min(ts + d.tile_elems, d.n);
      double* dst = W.part + (size_t)tile * WV_PAD;
      switch (ph) {
        case PH_ZERO: tile_zero<MB>(sh, d, ts, te, dst); break;
        case PH_STAGE1: tile_stage1<MB>(sh, d, ts, te, dst); break;
        case PH_CHECK: tile_check<MB>(sh, d, ts, te, dst); break;
        case PH_NEWTON: tile_newton<MB>(sh, d, ts, te, dst); break;
        default: tile_final<MB>(sh, d, ts, te, dst); break;
      }
    }
    trace_put(d, pass, 1, clk());
    trace_wg(d, pass, t_pass0, clk());
    if (!wide_sync(sh, d, W, pass, ph, nv)) break;
    trace_wg_go(d, pass, clk());
  }
  report_error(d, d.result ? &((pgdto_result*)d.result)->error : nullptr);
}

template <int MB>
__global__ __launch_bounds__(BLOCK, 1) void k_solve_wide(const Desc) {
  __shared__ ShW sh;
  __shared__ Desc sd;
  __shared__ int32_t late;
  load_desc(sd);
  if (!enter_launch(sd, &late)) return;
  solve_wide<MB>(sh, sd);
}

const void* wide_fn(int m) {
  switch ((m + 15) / 16) {
    case 1: return (const void*)k_solve_wide<1>;
    case 2: return (const void*)k_solve_wide<2>;
    case 3: return (const void*)k_solve_wide<3>;
    default: return (const void*)k_solve_wide<4>;
  }
}

}  // namespace pgdto
