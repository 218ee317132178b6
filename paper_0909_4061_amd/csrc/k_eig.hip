// The SVD of the small matrix B (Algorithm 5.1, step 2) for FP32 data, from
// the FP64 Gram W = B B* (l x l): the eigenvalues of W are the squared
// singular values of B and its eigenvectors are B's left singular vectors U~.
// For FP32 data this carries the accuracy of the Gram itself (relative error
// about u_64 (sigma_1 / sigma_j)^2 in sigma_j), well below what FP32 arithmetic
// resolves.  Three launches:
//
//   tridiag  : one workgroup.  Householder reduction W = Q_T T Q_T^T with T
//              symmetric tridiagonal.  The workgroup holds W in registers, a
//              2 x (l/16) tile per thread, 16 threads (one DPP row) per pair
//              of rows; step i takes its reflector from row i (the column by
//              symmetry), forms p = tau W v with 16-lane reductions, and
//              applies the symmetric rank-2 update W -= v w^T + w v^T.  Two
//              barriers per step (the reflector; the products p), with the
//              LDS vectors double-buffered.  Writes d, e, tau and the
//              reflectors.
//   tri_eig  : one wave per eigenvalue, four per workgroup.  Bisection on T
//              scaled to norm below one, by Sturm counts (three-term
//              recurrence of the leading minors, rescaled by powers of two)
//              at 64 points per round (one per lane): 9 rounds give 54 bits.
//              Then two steps of inverse iteration on T (LDL^T of T - lambda I
//              with tiny pivots lifted) from a pseudo-random start, the back
//              transform by the reflectors, and the outputs of this column.
//              An eigenvalue at the level of roundoff (|lambda| <= 64 eps ||T||)
//              or a failed solve keeps the random start and is flagged.
//   eig_fix  : one workgroup.  Eigenvalues closer than 2^-24 ||T|| form a
//              cluster: inverse iteration gives each member accurately within
//              the cluster's subspace but not orthogonal to the others, so the
//              members are orthogonalized in order (Gram-Schmidt, twice).
//              Flagged columns are orthogonalized against every other column
//              (a single flagged column becomes the missing eigenvector, since
//              the others span its complement).  Returns at once when no
//              column needs it.
#include <float.h>

#include <type_traits>

#include "common.hpp"

namespace rsvd {

namespace {

// Move a double across lanes of a 16-lane DPP row (every pattern used stays
// inside the row, so no lane reads out of bounds).
template <int CTRL>
__device__ __forceinline__ double eig_dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row; every lane ends with the same bits
// (each addition pairs the same two operands in all lanes).
__device__ __forceinline__ double row_sum16(double v) {
  v += eig_dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += eig_dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += eig_dpp<0x141>(v);  // row_half_mirror
  v += eig_dpp<0x140>(v);  // row_mirror
  return v;
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the whole wave, the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum16(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, eig_dpp<0x4E>(v));
  v = fmax(v, eig_dpp<0xB1>(v));
  v = fmax(v, eig_dpp<0x141>(v));
  v = fmax(v, eig_dpp<0x140>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Deterministic start vector of inverse iteration for eigenvalue j: a uniform
// value in [-1, 1) from an integer hash of (j, i).
__device__ __forceinline__ double start_value(int j, int i) {
  uint32_t h = (uint32_t)j * 0x9E3779B1u ^ ((uint32_t)i + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h >> 8) * 0x1p-23 - 1.0;
}

// ---------------------------------------------------------------------------
// tridiag: W -> (d, e, tau, reflectors).  NA groups of 16 lanes (one DPP row
// each); group a owns rows a + NA ri (ri < TR) and lane b of it columns
// b + 16 cc (cc < TC = MAXL / 16), both cyclic, so that the rows and columns
// that are done (index <= i at step i) leave every lane's tile at the same
// pace.  The steps run in segments of 16: in segment T (steps 16 T ..
// 16 T + 15) the column blocks cc < T and the row registers ri < RS = 16 T / NA
// hold only finished entries and are skipped at compile time, the reflector's
// row is register RS of group i mod NA, and only column block T (and the
// first lane of block T + 1) needs a mask.  Finished entries inside the live
// blocks are never read as data: v and p are zero there.
template <int MAXL>
constexpr int tri_groups() { return MAXL > 32 ? 32 : 16; }
template <int MAXL>
constexpr int tri_rows() { return MAXL / tri_groups<MAXL>(); }
template <int MAXL>
constexpr int tri_threads() { return tri_groups<MAXL>() * 16; }

// 1/sqrt(x) and 1/x from the hardware estimates and two Newton steps each.
__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// LDS vectors of the reduction, stored so that lane b of a group reads its TC
// columns b + 16 cc contiguously: entry c sits at (c mod 16) TC + c / 16.
template <int MAXL>
struct TriShared {
  double vbuf[2][MAXL];  // reflector v of the step (double-buffered)
  double pbuf[2][MAXL];  // p = tau W v
  double kpart[2][32];   // per group: sum of p_r v_r over its rows
  double taus[2];
};

template <int MAXL, int T>
__device__ __forceinline__ void tridiag_segment(const EigParams& p, TriShared<MAXL>& sh,
                                                double (&w)[tri_rows<MAXL>()][MAXL / 16], int nsteps) {
  constexpr int TR = tri_rows<MAXL>(), TC = MAXL / 16, NA = tri_groups<MAXL>();
  constexpr int RS = 16 * T / NA;  // first live row register
  constexpr int RSTEP = NA / 16;   // position stride of a group's successive rows
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, a = tid >> 4, b = tid & 15, lane = tid & 63;
  const int l = p.l;
  const int rp0 = (a & 15) * TC + (a >> 4);  // position of row a
  const int iend = min(16 * T + 16, nsteps);
  for (int i = 16 * T; i < iend; ++i) {
    const int buf = i & 1, ib = i - 16 * T;
    // 1. reflector of row i (= column i) by group i mod NA from its register RS
    if (a == (i & (NA - 1))) {
      const int gl = 16 * ((i & (NA - 1)) & 3);  // first lane of the group in its wave
      const double xt = w[RS][T];
      const double xn = T + 1 < TC ? w[RS][T + 1 < TC ? T + 1 : T] : 0.0;
      const double dii = lane_value(xt, gl + ib);
      const double x0 = ib < 15 ? lane_value(xt, gl + min(ib + 1, 15)) : lane_value(xn, gl);
      const bool mt = b >= ib + 2;             // block T: column >= i + 2
      const bool mn = ib < 15 || b > 0;        // block T + 1: column >= i + 2
      double s2 = mt ? xt * xt : 0.0;
      if (T + 1 < TC) s2 = mn ? fma(xn, xn, s2) : s2;
#pragma unroll
      for (int cc = T + 2; cc < TC; ++cc) s2 = fma(w[RS][cc], w[RS][cc], s2);
      s2 = row_sum16(s2);
      double tau = 0.0, beta = x0, scal = 0.0;
      if (s2 > 0.0) {
        const double n2 = fma(x0, x0, s2);
        const double rn = rsq_refined(n2);   // 1 / ||x||
        const double nrm = n2 * rn;          // ||x||
        beta = x0 >= 0.0 ? -nrm : nrm;       // -sign(x0) ||x||
        tau = fma(x0, x0 >= 0.0 ? rn : -rn, 1.0);  // (beta - x0) / beta = 1 - x0 / beta
        scal = rcp_refined(x0 - beta);
      }
      double v[TC];
#pragma unroll
      for (int cc = 0; cc < TC; ++cc) v[cc] = cc > T + 1 ? w[RS][cc] * scal : 0.0;
      v[T] = mt ? xt * scal : (b == ib + 1 ? 1.0 : 0.0);
      if (T + 1 < TC) v[T + 1 < TC ? T + 1 : T] = mn ? xn * scal : 1.0;
#pragma unroll
      for (int cc = 0; cc < TC; cc += 2) *reinterpret_cast<d2*>(&sh.vbuf[buf][b * TC + cc]) = d2{v[cc], v[cc + 1]};
      double* vrow = p.V + (int64_t)i * EIG_LDV + b;
#pragma unroll
      for (int cc = 0; cc < TC; ++cc) vrow[16 * cc] = v[cc];
      if (b == 0) {
        sh.taus[buf] = tau;
        p.tri[i] = dii;
        p.tri[l + i] = beta;
        p.tri[2 * l + i] = tau;
      }
    }
    __syncthreads();
    // 2. p = tau W v (rows <= i give zero), and this group's share of p.v
    const double tau = sh.taus[buf];
    double vr[TR], pr[TR], vc[TC];
#pragma unroll
    for (int ri = RS; ri < TR; ++ri) vr[ri] = sh.vbuf[buf][rp0 + RSTEP * ri];
#pragma unroll
    for (int cc = T & ~1; cc < TC; cc += 2) {
      const d2 t = *reinterpret_cast<const d2*>(&sh.vbuf[buf][b * TC + cc]);
      vc[cc] = t.x;
      vc[cc + 1] = t.y;
    }
    double kp = 0.0;
#pragma unroll
    for (int ri = RS; ri < TR; ++ri) {
      double s = 0.0;
#pragma unroll
      for (int cc = T; cc < TC; ++cc) s = fma(w[ri][cc], vc[cc], s);
      s = row_sum16(s) * tau;
      if (ri == RS) s = a + NA * RS > i ? s : 0.0;
      pr[ri] = s;
      kp = fma(s, vr[ri], kp);
    }
    if (b == 0) {
#pragma unroll
      for (int ri = RS; ri < TR; ++ri) sh.pbuf[buf][rp0 + RSTEP * ri] = pr[ri];
      sh.kpart[buf][a] = kp;
    }
    __syncthreads();
    // 3. K = tau/2 p.v, w = p - K v, W -= v w^T + w v^T over the live tile
    const double K = 0.5 * tau * wave_sum(lane < NA ? sh.kpart[buf][lane] : 0.0);
    double wr[TR];
#pragma unroll
    for (int ri = RS; ri < TR; ++ri) wr[ri] = fma(-K, vr[ri], pr[ri]);
#pragma unroll
    for (int cc = T & ~1; cc < TC; cc += 2) {
      const d2 t = *reinterpret_cast<const d2*>(&sh.pbuf[buf][b * TC + cc]);
      const double pc[2] = {t.x, t.y};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (cc + h < T) continue;
        const double wc = fma(-K, vc[cc + h], pc[h]);
#pragma unroll
        for (int ri = RS; ri < TR; ++ri) w[ri][cc + h] = fma(-vr[ri], wc, fma(-wr[ri], vc[cc + h], w[ri][cc + h]));
      }
    }
  }
  if constexpr (T + 1 < MAXL / 16) {
    if (16 * (T + 1) < nsteps) tridiag_segment<MAXL, T + 1>(p, sh, w, nsteps);
  }
}

template <int MAXL>
__device__ __forceinline__ void tridiag_body(const EigParams& p) {
  constexpr int TR = tri_rows<MAXL>(), TC = MAXL / 16, NA = tri_groups<MAXL>();
  static_assert(MAXL % 16 == 0 && TC % 2 == 0 && (NA == 16 || NA == 32) && TR * NA == MAXL, "tile layout");
  __shared__ __attribute__((aligned(16))) TriShared<MAXL> sh;
  const int tid = threadIdx.x, a = tid >> 4, b = tid & 15;
  const int l = p.l, Lg = p.Lg;
  double w[TR][TC];
#pragma unroll
  for (int ri = 0; ri < TR; ++ri)
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) {
      const int r = a + NA * ri, c = b + 16 * cc;
      w[ri][cc] = (r < l && c < l) ? p.G[(int64_t)min(r, c) * Lg + max(r, c)] : 0.0;
    }
  const int nsteps = l > 2 ? l - 2 : 0;
  if (nsteps > 0) tridiag_segment<MAXL, 0>(p, sh, w, nsteps);
  // the last 2 x 2 block (or 1 x 1) is already tridiagonal
#pragma unroll
  for (int ri = 0; ri < TR; ++ri)
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) {
      const int r = a + NA * ri, c = b + 16 * cc;
      if (r < l && r >= l - 2 && c == r) p.tri[r] = w[ri][cc];
      if (l >= 2 && r == l - 2 && c == l - 1) p.tri[l + l - 2] = w[ri][cc];
    }
  if (tid == 0) {
    if (l >= 1) p.tri[l + l - 1] = 0.0;
    for (int i = max(l - 2, 0); i < l; ++i) p.tri[2 * l + i] = 0.0;
  }
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dbl2 ld2(const double* p) { return *reinterpret_cast<const dbl2*>(p); }

// The vectors of the scaled T's recurrences live in registers: register b of
// lane k holds entry 16 b + (k mod 16), the same in each of the wave's four
// 16-lane rows, and entry 16 b + c reaches every lane by one 64-bit DPP
// broadcast of lane c of the row.  The recurrences, which every lane runs with
// its own shift, read no memory.
template <int NB>
struct TriReg {
  double r[NB];
};

template <int NB>
__device__ __forceinline__ TriReg<NB> tri_load(const double* __restrict__ v, int lane) {
  TriReg<NB> t;
#pragma unroll
  for (int b = 0; b < NB; ++b) t.r[b] = v[16 * b + (lane & 15)];
  return t;
}

template <int C>
__device__ __forceinline__ double eig_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, false);  // row_newbcast: lane C of the row
}

// f(std::integral_constant<int, c>) for c = C .. 15, or 15 down to C when DOWN.
template <int C, bool DOWN = false, typename F>
__device__ __forceinline__ void for16(F&& f) {
  if constexpr (C < 16) {
    if constexpr (DOWN) {
      for16<C + 1, DOWN>(f);
      f(std::integral_constant<int, C>{});
    } else {
      f(std::integral_constant<int, C>{});
      for16<C + 1, DOWN>(f);
    }
  }
}

// Number of eigenvalues of the scaled T below x: sign changes of the leading
// minors p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}, rescaled by a power of two
// every four steps.  A zero minor counts as non-negative: with e_i^2 > 0 the
// minor after it is -e_i^2 times the one before it, so exactly one sign change
// falls on the pair around the zero whichever sign the zero is given.  The
// recurrence runs over whole blocks of 16 (nblk of them); past l the diagonal
// holds 4 > |x|, which changes no count.
template <int NB>
__device__ __forceinline__ int sturm_count(const TriReg<NB>& dr, const TriReg<NB>& e2r, int nblk, double x) {
  double pm2 = 0.0, pm1 = 1.0;
  int cnt = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b >= nblk) break;
    for16<0>([&](auto ci) {
      constexpr int c = decltype(ci)::value;
      const double pi = fma(eig_bcast<c>(dr.r[b]) - x, pm1, -eig_bcast<c>(e2r.r[b]) * pm2);
      cnt += (pi < 0.0) != (pm1 < 0.0) ? 1 : 0;
      pm2 = pm1;
      pm1 = pi;
      if constexpr (c % 4 == 3) {
        const int ex = __builtin_amdgcn_frexp_exp(pm1);
        pm1 = __builtin_amdgcn_ldexp(pm1, -ex);
        pm2 = __builtin_amdgcn_ldexp(pm2, -ex);
      }
    });
  }
  return cnt;
}

// tri_eig: eigenpair j = 4 blockIdx + wave (descending order) of T, then of W.
// STAGE: the reflectors of the back transform are staged in LDS (MAXL^2
// doubles) once for the workgroup's four waves -- for a single matrix, whose
// few workgroups then wait on no global loads; a batch of many matrices keeps
// the LDS small (more workgroups per CU) and reads them from global memory one
// reflector ahead.
template <int MAXL, bool STAGE>
__device__ __forceinline__ void tri_eig_body(const EigParams& p, const int bid) {
  __shared__ __attribute__((aligned(16))) double ds[MAXL];   // scaled diagonal (4.0 past l)
  __shared__ __attribute__((aligned(16))) double es[MAXL];   // scaled off-diagonal, es[i] couples i and i + 1
  __shared__ __attribute__((aligned(16))) double e2p[MAXL];  // es[i - 1]^2 (0 for i = 0)
  __shared__ __attribute__((aligned(16))) double invD[4][MAXL];
  __shared__ __attribute__((aligned(16))) double Lm[4][MAXL];
  __shared__ __attribute__((aligned(16))) double xs[4][MAXL];
  __shared__ __attribute__((aligned(16))) double Vs[STAGE ? MAXL * MAXL : 2];  // reflector i at Vs[i * MAXL]
  __shared__ double ts[MAXL];                                                  // tau
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = p.l;
  const double* __restrict__ dvec = p.tri;
  const double* __restrict__ evec = p.tri + l;
  const double* __restrict__ tvec = p.tri + 2 * l;
  for (int i = tid; i < MAXL; i += 256) {
    ds[i] = i < l ? dvec[i] : 0.0;
    es[i] = i + 1 < l ? evec[i] : 0.0;
  }
  for (int i = tid; i < MAXL; i += 256) ts[i] = i < l ? tvec[i] : 0.0;
  // the reflectors of the back transform, staged once for the workgroup's four waves
  if (STAGE) {
    const dbl2* __restrict__ src = reinterpret_cast<const dbl2*>(p.V);
    constexpr int PER_ROW = MAXL / 2;
    for (int q = tid; q < (l - 2 > 0 ? l - 2 : 0) * PER_ROW; q += 256) {
      const int r = q / PER_ROW, c2 = q - r * PER_ROW;
      *reinterpret_cast<dbl2*>(Vs + r * MAXL + 2 * c2) = src[(int64_t)r * (EIG_LDV / 2) + c2];
    }
  }
  __syncthreads();
  // ||T|| bound (Gershgorin) and its power-of-two scale, the same in every wave
  double g = 0.0;
  for (int i = lane; i < l; i += 64) g = fmax(g, fabs(ds[i]) + fabs(es[i]) + (i > 0 ? fabs(es[i - 1]) : 0.0));
  const double tnorm = wave_max(g);
  const int tex = tnorm > 0.0 ? __builtin_amdgcn_frexp_exp(tnorm) : 0;
  __syncthreads();  // every wave has read the unscaled values
  for (int i = tid; i < MAXL; i += 256) {
    ds[i] = i < l ? __builtin_amdgcn_ldexp(ds[i], -tex) : 4.0;
    es[i] = __builtin_amdgcn_ldexp(es[i], -tex);
  }
  __syncthreads();
  // e^2 floored at 2^-200 (eigenvalues move by at most 2^-100 of ||T||): no
  // coupling is exactly zero, so a zero minor is always followed by a nonzero one
  for (int i = tid; i < MAXL; i += 256) e2p[i] = i > 0 ? fmax(es[i - 1] * es[i - 1], 0x1p-200) : 0.0;
  __syncthreads();
  const int j = 4 * bid + wv;
  if (j >= l) return;
  constexpr int NB = MAXL / 16;
  const int nblk = (l + 15) >> 4;  // the recurrences run over whole blocks of 16
  const TriReg<NB> dr = tri_load<NB>(ds, lane), er = tri_load<NB>(es, lane), e2r = tri_load<NB>(e2p, lane);
  if (bid == 0 && tid == 0) p.tnorm[0] = tnorm;

  // 1. bisection for the (l - 1 - j)-th smallest eigenvalue of the scaled T
  double glo = 0.0, ghi = 0.0;
  {
    double lo = 1.0, hi = -1.0;
    for (int i = lane; i < l; i += 64) {
      const double r = fabs(es[i]) + (i > 0 ? fabs(es[i - 1]) : 0.0);
      lo = fmin(lo, ds[i] - r);
      hi = fmax(hi, ds[i] + r);
    }
    glo = -wave_max(-lo);
    ghi = wave_max(hi);
  }
  const double slack = 4.0 * DBL_EPSILON * fmax(fabs(glo), fabs(ghi)) + DBL_MIN;
  double lo = glo - slack, hi = ghi + slack;
  const int jasc = l - 1 - j;
  const double frac = (double)(lane + 1) * (1.0 / 65.0);
  for (int round = 0; round < 9; ++round) {
    const double wdt = hi - lo;
    const double x = fma(wdt, frac, lo);
    const int cnt = tnorm > 0.0 ? sturm_count<NB>(dr, e2r, nblk, x) : (x > 0.0 ? l : 0);
    const uint64_t mask = __ballot(cnt <= jasc);
    const int m = __popcll(mask) - 1;  // last point at or below the eigenvalue
    const double nlo = m >= 0 ? fma(wdt, (double)(m + 1) * (1.0 / 65.0), lo) : lo;
    const double nhi = m + 1 <= 63 ? fma(wdt, (double)(m + 2) * (1.0 / 65.0), lo) : hi;
    lo = nlo;
    hi = nhi;
  }
  const double mu = 0.5 * (lo + hi);
  const double lam = __builtin_amdgcn_ldexp(mu, tex);

  // 2. inverse iteration (every lane runs the scalar recurrences; the stores agree)
  double* __restrict__ iD = invD[wv];
  double* __restrict__ L = Lm[wv];
  double* __restrict__ x = xs[wv];
  bool flagged = !(fabs(mu) > 64.0 * DBL_EPSILON);
  for (int i = lane; i < MAXL; i += 64) x[i] = i < l ? start_value(j, i) : 0.0;
  if (!flagged) {
    // LDL^T of the scaled T - mu I over whole blocks of 16 (the rows past l
    // decouple: e = 0), tiny pivots lifted to +-2^-62.  Every lane runs the
    // recurrences and stores the same values; each pass reads its inputs from
    // registers and the next pass reloads its outputs from LDS.
    const double ptol = 0x1p-62;
    {
      double inv = 0.0, eprev = 0.0, li4[4], iv4[4];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b >= nblk) break;
        for16<0>([&](auto ci) {
          constexpr int c = decltype(ci)::value;
          const double li = eprev * inv;  // 0 at i = 0 (eprev = 0)
          double D = fma(-li, eprev, eig_bcast<c>(dr.r[b]) - mu);
          D = fabs(D) < ptol ? (D < 0.0 ? -ptol : ptol) : D;
          inv = rcp_refined(D);
          li4[c % 4] = li;
          iv4[c % 4] = inv;
          eprev = eig_bcast<c>(er.r[b]);
          if constexpr (c % 4 == 3) {
            const int i0 = 16 * b + c - 3;
            *reinterpret_cast<dbl2*>(iD + i0) = dbl2{iv4[0], iv4[1]};
            *reinterpret_cast<dbl2*>(iD + i0 + 2) = dbl2{iv4[2], iv4[3]};
            *reinterpret_cast<dbl2*>(L + i0) = dbl2{li4[0], li4[1]};
            *reinterpret_cast<dbl2*>(L + i0 + 2) = dbl2{li4[2], li4[3]};
          }
        });
      }
    }
    const TriReg<NB> Lr = tri_load<NB>(L, lane), iDr = tri_load<NB>(iD, lane);
    for (int it = 0; it < 2; ++it) {
      // L y = x (forward), then D L^T x = y (backward), in place
      {
        const TriReg<NB> xr = tri_load<NB>(x, lane);
        double y = 0.0, y4[4];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (b >= nblk) break;
          for16<0>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            y = fma(-eig_bcast<c>(Lr.r[b]), y, eig_bcast<c>(xr.r[b]));  // L[0] = 0
            y4[c % 4] = y;
            if constexpr (c % 4 == 3) {
              const int i0 = 16 * b + c - 3;
              *reinterpret_cast<dbl2*>(x + i0) = dbl2{y4[0], y4[1]};
              *reinterpret_cast<dbl2*>(x + i0 + 2) = dbl2{y4[2], y4[3]};
            }
          });
        }
      }
      // x_i = y_i / D_i - L_{i+1} x_{i+1}, from the last row of the last block down
      // (L past it taken as 0)
      {
        const TriReg<NB> yr = tri_load<NB>(x, lane);
        double xn = 0.0, lnext = 0.0, x4[4];
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
          const int b = NB - 1 - bb;
          if (b >= nblk) continue;
          for16<0, true>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            xn = fma(-lnext, xn, eig_bcast<c>(yr.r[b]) * eig_bcast<c>(iDr.r[b]));
            x4[c % 4] = xn;
            lnext = eig_bcast<c>(Lr.r[b]);
            if constexpr (c % 4 == 0) {
              const int i0 = 16 * b + c;
              *reinterpret_cast<dbl2*>(x + i0) = dbl2{x4[0], x4[1]};
              *reinterpret_cast<dbl2*>(x + i0 + 2) = dbl2{x4[2], x4[3]};
            }
          });
        }
      }
      double s = 0.0;
      for (int i = lane; i < l; i += 64) s = fma(x[i], x[i], s);
      s = wave_sum(s);
      if (!(s > 0.0) || !isfinite(s)) {
        flagged = true;
        break;
      }
      const double sc = 1.0 / sqrt(s);
      for (int i = lane; i < l; i += 64) x[i] *= sc;
    }
    if (flagged)
      for (int i = lane; i < MAXL; i += 64) x[i] = i < l ? start_value(j, i) : 0.0;
  }
  // 3. back transform z = H_0 H_1 ... H_{l-3} x (normalized)
  double z0 = lane < l ? x[lane] : 0.0;
  double z1 = lane + 64 < l ? x[lane + 64] : 0.0;
  if (flagged) {
    const double s = wave_sum(z0 * z0 + z1 * z1);
    const double sc = 1.0 / sqrt(s);
    z0 *= sc;
    z1 *= sc;
  }
  // (columns at or past l of a reflector row are masked)
  if (STAGE) {
    for (int i = l - 3; i >= 0; --i) {
      const double v0 = lane < l ? Vs[i * MAXL + lane] : 0.0;
      const double v1 = lane + 64 < l ? Vs[i * MAXL + (lane + 64 < MAXL ? lane + 64 : 0)] : 0.0;
      const double dot = wave_sum(fma(v0, z0, v1 * z1)) * ts[i];
      z0 = fma(-dot, v0, z0);
      z1 = fma(-dot, v1, z1);
    }
  } else if (l >= 3) {
    const double* __restrict__ V = p.V;
    double v0 = lane < l ? V[(int64_t)(l - 3) * EIG_LDV + lane] : 0.0;
    double v1 = lane + 64 < l ? V[(int64_t)(l - 3) * EIG_LDV + lane + 64] : 0.0;
    for (int i = l - 3; i >= 0; --i) {
      const int ni = i > 0 ? i - 1 : 0;
      const double n0 = lane < l ? V[(int64_t)ni * EIG_LDV + lane] : 0.0;
      const double n1 = lane + 64 < l ? V[(int64_t)ni * EIG_LDV + lane + 64] : 0.0;
      const double dot = wave_sum(fma(v0, z0, v1 * z1)) * ts[i];
      z0 = fma(-dot, v0, z0);
      z1 = fma(-dot, v1, z1);
      v0 = n0;
      v1 = n1;
    }
  }
  // 4. the sign convention of the small SVD (also the Jacobi kernel's): the
  //    component of largest magnitude, the first of equals, is positive
  {
    const double a0 = lane < l ? fabs(z0) : -1.0, a1 = lane + 64 < l ? fabs(z1) : -1.0;
    const double mx = wave_max(fmax(a0, a1));
    const uint64_t b0 = __ballot(a0 == mx), b1 = __ballot(a1 == mx);
    const int at = b0 ? __ffsll((long long)b0) - 1 : 64 + __ffsll((long long)b1) - 1;
    const double piv = at < 64 ? lane_value(z0, at) : lane_value(z1, at - 64);
    if (piv < 0.0) {
      z0 = -z0;
      z1 = -z1;
    }
  }
  // 5. this column's outputs
  const double sg = sqrt(fmax(lam, 0.0));
  if (lane == 0) {
    p.lam[j] = lam;
    p.flag[j] = flagged ? 1 : 0;
    p.sig[j] = sg;
    if (j < p.k) {
      if (p.dtype == RSVD_F64) ((double*)p.S)[j] = sg;
      else ((float*)p.S)[j] = (float)sg;
    }
  }
  const double rs = sg > 0.0 ? 1.0 / sg : 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
    const double zi = h ? z1 : z0;
    if (i < l) {
      p.Z[(int64_t)j * l + i] = zi;
      p.Uh[(int64_t)i * l + j] = zi;
      if (j < p.k) {
        if (p.dtype == RSVD_F64) {
          ((double*)p.XU)[(int64_t)i * p.k + j] = zi;
          ((double*)p.XV)[(int64_t)i * p.k + j] = zi * rs;
        } else {
          ((float*)p.XU)[(int64_t)i * p.k + j] = (float)zi;
          ((float*)p.XV)[(int64_t)i * p.k + j] = (float)(zi * rs);
        }
      }
    }
  }
}

// eig_fix: one workgroup of 256 threads.  Column c of Zs holds eigenvector c.
template <int MAXL>
__device__ __forceinline__ void eig_fix_body(const EigParams& p) {
  constexpr int LDZ = MAXL + 2;       // even: 16-byte aligned columns
  constexpr int HALF = MAXL / 2;
  __shared__ __attribute__((aligned(16))) double Zs[MAXL * LDZ];  // Zs[c * LDZ + i] = component i of vector c (0 past l)
  __shared__ __attribute__((aligned(16))) double coef[MAXL];
  __shared__ int todo[MAXL];         // 0 keep, 1 cluster member after the first, 2 flagged
  __shared__ int clu0[MAXL];         // first member of the vector's cluster
  __shared__ double lam_s[MAXL];
  __shared__ int any_s;
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = p.l;
  for (int j = tid; j < l; j += 256) {
    lam_s[j] = p.lam[j];
    todo[j] = p.flag[j];
  }
  __syncthreads();
  if (tid == 0) {
    const double tol = 0x1p-24 * p.tnorm[0];
    int any = 0, first = 0;
    for (int j = 0; j < l; ++j) {
      if (j > 0 && !(lam_s[j - 1] - lam_s[j] >= tol)) {
        clu0[j] = first;
      } else {
        first = j;
        clu0[j] = j;
      }
      const int t = todo[j] ? 2 : (clu0[j] != j ? 1 : 0);
      todo[j] = t;
      any |= t;
    }
    any_s = any;
  }
  __syncthreads();
  if (!any_s) return;
  for (int idx = tid; idx < MAXL * MAXL; idx += 256) {
    const int c = idx / MAXL, i = idx - c * MAXL;
    Zs[c * LDZ + i] = (c < l && i < l) ? p.Z[(int64_t)c * l + i] : 0.0;
  }
  __syncthreads();
  // phase 1 (clusters, flagged columns left out), then phase 2 (flagged columns)
  for (int phase = 1; phase <= 2; ++phase) {
    for (int j = 0; j < l; ++j) {
      if (todo[j] != phase) continue;  // uniform
      for (int attempt = 0; attempt < 2 * MAXL; ++attempt) {
        for (int rep = 0; rep < 2; ++rep) {
          // coefficients against the columns this one must be orthogonal to: thread
          // pair (2 c, 2 c + 1) takes the two halves of the dot product with column c
          {
            const int c = tid >> 1, h = tid & 1;
            bool use = false;
            if (c < l) {
              if (phase == 1) use = c >= clu0[j] && c < j && todo[c] != 2;
              else use = c != j && (todo[c] != 2 || c < j);
            }
            // (fixed trip count over the padded half, four partial sums, 16-byte reads)
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            if (use) {
              const double* zc = Zs + c * LDZ + h * HALF;
              const double* zj = Zs + j * LDZ + h * HALF;
#pragma unroll
              for (int q = 0; q < HALF; q += 2) {
                const dbl2 x = *reinterpret_cast<const dbl2*>(zc + q), y = *reinterpret_cast<const dbl2*>(zj + q);
                s4[q & 2] = fma(x.x, y.x, s4[q & 2]);
                s4[(q & 2) + 1] = fma(x.y, y.y, s4[(q & 2) + 1]);
              }
            }
            double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            s += eig_dpp<0xB1>(s);  // quad_perm [1,0,3,2]: the partner's half
            if (c < MAXL && h == 0) coef[c] = s;
          }
          __syncthreads();
          {
            const int i = tid >> 1, h = tid & 1;
            double s4[4] = {0.0, 0.0, 0.0, 0.0};  // coef is zero for the columns not used
            // only the columns that can have a nonzero coefficient ([clu0[j], j) in phase 1), in
            // steps of four from a multiple of four: each term keeps its partial sum and the skipped
            // terms were exact zeros, so the sums are the ones of the full loop
            const int clo = phase == 1 ? clu0[j] : 0, chi = phase == 1 ? j : l;
            const int qlo = max(0, (clo - h * HALF) & ~3), qhi = min(HALF, ((chi - h * HALF) + 3) & ~3);
            if (i < l) {
              for (int q = qlo; q < qhi; q += 4) {
#pragma unroll
                for (int u = 0; u < 4; u += 2) {
                  const int c = h * HALF + q + u;
                  const dbl2 cf = *reinterpret_cast<const dbl2*>(coef + c);
                  s4[u] = fma(-cf.x, Zs[c * LDZ + i], s4[u]);
                  s4[u + 1] = fma(-cf.y, Zs[(c + 1) * LDZ + i], s4[u + 1]);
                }
              }
            }
            double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            s += eig_dpp<0xB1>(s);
            __syncthreads();  // every thread has read column j for its coefficient before it changes
            if (i < l && h == 0) Zs[j * LDZ + i] += s;
          }
          __syncthreads();
        }
        double s = 0.0;
        for (int i = tid; i < l; i += 256) s = fma(Zs[j * LDZ + i], Zs[j * LDZ + i], s);
        s = wave_sum(s);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        const double nrm2 = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
        // Two Gram-Schmidt passes leave the column orthogonal to the others to working
        // precision unless nearly all of it was cancelled; a random column keeps about
        // (l - #others) / l of its squared norm, at least 1 / l.
        if (nrm2 > 0x1p-20) {
          const double sc = 1.0 / sqrt(nrm2);
          for (int i = tid; i < l; i += 256) Zs[j * LDZ + i] *= sc;
          __syncthreads();
          break;
        }
        // the column lay (almost) in the span of the others: restart from a unit vector
        for (int i = tid; i < l; i += 256) Zs[j * LDZ + i] = (i == attempt % l) ? 1.0 : 0.0;
        __syncthreads();
      }
    }
  }
  // outputs of the columns that changed, with the sign convention of tri_eig
  for (int j = tid; j < l; j += 256) {
    if (todo[j] == 0) continue;
    double mx = -1.0, piv = 1.0;
    for (int i = 0; i < l; ++i) {
      const double v = Zs[j * LDZ + i];
      if (fabs(v) > mx) {
        mx = fabs(v);
        piv = v;
      }
    }
    coef[j] = piv < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < l * l; idx += 256) {
    const int j = idx / l, i = idx - j * l;
    if (todo[j] == 0) continue;
    const double zi = coef[j] * Zs[j * LDZ + i];
    p.Uh[(int64_t)i * l + j] = zi;
    if (j < p.k) {
      const double sg = p.sig[j];
      const double rs = sg > 0.0 ? 1.0 / sg : 0.0;
      if (p.dtype == RSVD_F64) {
        ((double*)p.XU)[(int64_t)i * p.k + j] = zi;
        ((double*)p.XV)[(int64_t)i * p.k + j] = zi * rs;
      } else {
        ((float*)p.XU)[(int64_t)i * p.k + j] = (float)zi;
        ((float*)p.XV)[(int64_t)i * p.k + j] = (float)(zi * rs);
      }
    }
  }
}

template <int MAXL>
__global__ __launch_bounds__(tri_threads<MAXL>()) void tridiag_kernel(const EigParams p) { tridiag_body<MAXL>(p); }

template <int MAXL>
__global__ __launch_bounds__(tri_threads<MAXL>()) void tridiag_batched(const EigParams* __restrict__ ps,
                                                                     const BlockMap* __restrict__ bm) {
  tridiag_body<MAXL>(ps[bm[blockIdx.x].item]);
}

template <int MAXL>
__global__ __launch_bounds__(256) void tri_eig_kernel(const EigParams p) { tri_eig_body<MAXL, true>(p, blockIdx.x); }

template <int MAXL>
__global__ __launch_bounds__(256) void tri_eig_batched(const EigParams* __restrict__ ps,
                                                      const BlockMap* __restrict__ bm) {
  const BlockMap b = bm[blockIdx.x];
  tri_eig_body<MAXL, false>(ps[b.item], b.local);
}

template <int MAXL>
__global__ __launch_bounds__(256) void eig_fix_kernel(const EigParams p) { eig_fix_body<MAXL>(p); }

template <int MAXL>
__global__ __launch_bounds__(256) void eig_fix_batched(const EigParams* __restrict__ ps,
                                                      const BlockMap* __restrict__ bm) {
  eig_fix_body<MAXL>(ps[bm[blockIdx.x].item]);
}

// Two independent problems of one size in one launch per stage (both parameter
// sets by value): blocks [0, nb0) serve the first, the rest the second.
template <int MAXL>
__global__ __launch_bounds__(tri_threads<MAXL>()) void tridiag_pair(const EigParams p0, const EigParams p1) {
  if (blockIdx.x == 0)
    tridiag_body<MAXL>(p0);
  else
    tridiag_body<MAXL>(p1);
}

template <int MAXL>
__global__ __launch_bounds__(256) void tri_eig_pair(const EigParams p0, const EigParams p1, const int nb0) {
  const int b = (int)blockIdx.x;
  if (b < nb0)
    tri_eig_body<MAXL, true>(p0, b);
  else
    tri_eig_body<MAXL, true>(p1, b - nb0);
}

template <int MAXL>
__global__ __launch_bounds__(256) void eig_fix_pair(const EigParams p0, const EigParams p1) {
  if (blockIdx.x == 0)
    eig_fix_body<MAXL>(p0);
  else
    eig_fix_body<MAXL>(p1);
}

bool eig_params_ok(const EigParams& p) {
  return p.l >= 1 && p.l <= 128 && p.k >= 1 && p.k <= p.l && p.Lg >= p.l;
}

}  // namespace

int eig_variant(int32_t l) { return l <= 32 ? 32 : (l <= 64 ? 64 : (l <= 96 ? 96 : 128)); }

int64_t tri_eig_blocks(const EigParams& p) { return (p.l + 3) / 4; }

#define RSVD_EIG_SWITCH(VAR, CALL)              \
  switch (VAR) {                                \
    case 32: CALL(32); break;                   \
    case 64: CALL(64); break;                   \
    case 96: CALL(96); break;                   \
    case 128: CALL(128); break;                 \
    default: return hipErrorInvalidValue;       \
  }

int64_t eig_blocks(int stage, const EigParams& p) { return stage == 1 ? tri_eig_blocks(p) : 1; }

hipError_t launch_eig(int stage, const EigParams& p, hipStream_t st) {
  if (!eig_params_ok(p) || stage < 0 || stage > 2) return hipErrorInvalidValue;
  const int v = eig_variant(p.l);
  const dim3 g2((unsigned)tri_eig_blocks(p));
#define RSVD_L1(M) hipLaunchKernelGGL(tridiag_kernel<M>, dim3(1), dim3(tri_threads<M>()), 0, st, p)
#define RSVD_L2(M) hipLaunchKernelGGL(tri_eig_kernel<M>, g2, dim3(256), 0, st, p)
#define RSVD_L3(M) hipLaunchKernelGGL(eig_fix_kernel<M>, dim3(1), dim3(256), 0, st, p)
  if (stage == 0) {
    RSVD_EIG_SWITCH(v, RSVD_L1)
  } else if (stage == 1) {
    RSVD_EIG_SWITCH(v, RSVD_L2)
  } else {
    RSVD_EIG_SWITCH(v, RSVD_L3)
  }
#undef RSVD_L1
#undef RSVD_L2
#undef RSVD_L3
  return hipGetLastError();
}

hipError_t launch_eig_pair(int stage, const EigParams& a, const EigParams& b, hipStream_t st) {
  if (!eig_params_ok(a) || !eig_params_ok(b) || a.l != b.l || stage < 0 || stage > 2) return hipErrorInvalidValue;
  const int v = eig_variant(a.l);
  const int nb0 = (int)tri_eig_blocks(a);
  const dim3 g2((unsigned)(nb0 + tri_eig_blocks(b)));
#define RSVD_P1(M) hipLaunchKernelGGL(tridiag_pair<M>, dim3(2), dim3(tri_threads<M>()), 0, st, a, b)
#define RSVD_P2(M) hipLaunchKernelGGL(tri_eig_pair<M>, g2, dim3(256), 0, st, a, b, nb0)
#define RSVD_P3(M) hipLaunchKernelGGL(eig_fix_pair<M>, dim3(2), dim3(256), 0, st, a, b)
  if (stage == 0) {
    RSVD_EIG_SWITCH(v, RSVD_P1)
  } else if (stage == 1) {
    RSVD_EIG_SWITCH(v, RSVD_P2)
  } else {
    RSVD_EIG_SWITCH(v, RSVD_P3)
  }
#undef RSVD_P1
#undef RSVD_P2
#undef RSVD_P3
  return hipGetLastError();
}

hipError_t launch_eig_batched(int stage, int variant, const EigParams* ps, const BlockMap* bm, int64_t nblocks,
                              hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 g((unsigned)nblocks);
#define RSVD_B1(M) hipLaunchKernelGGL(tridiag_batched<M>, g, dim3(tri_threads<M>()), 0, st, ps, bm)
#define RSVD_B2(M) hipLaunchKernelGGL(tri_eig_batched<M>, g, dim3(256), 0, st, ps, bm)
#define RSVD_B3(M) hipLaunchKernelGGL(eig_fix_batched<M>, g, dim3(256), 0, st, ps, bm)
  if (stage == 0) {
    RSVD_EIG_SWITCH(variant, RSVD_B1)
  } else if (stage == 1) {
    RSVD_EIG_SWITCH(variant, RSVD_B2)
  } else {
    RSVD_EIG_SWITCH(variant, RSVD_B3)
  }
#undef RSVD_B1
#undef RSVD_B2
#undef RSVD_B3
  return hipGetLastError();
}

}  // namespace rsvd
