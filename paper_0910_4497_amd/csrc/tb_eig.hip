// Projected eigenproblem and density-matrix assembly (Sec. 3: the small
// projected matrix is diagonalised; Sec. 2, Eq. 2: rho = sum |m> f <m|).
//
// k_band (one wave per atom) and k_eig (one persistent workgroup per atom at
// a time), FP64:
//   1. k_band: T (block tridiagonal, 4x4 blocks A_k, upper-triangular B_k: a
//      band of half-width 4) -> tridiagonal S = Z^T T Z by Householder
//      reflectors of length 4 with bulge chasing. Sweep j annihilates
//      column j below its subdiagonal with a reflector on rows j+1..j+4;
//      applied from both sides it fills a 4x4 bulge below the window, whose
//      first column the sweep's next task annihilates with a reflector four
//      rows further down, and so on to the end of the matrix (the fill stays
//      within seven diagonals below the main one). Task (j, s) is the s-th of
//      sweep j, its window at row p0 = j + 1 + 4 s; it runs at time step
//      3 j + s, so the tasks of one step are 11 rows apart and touch
//      disjoint entries: each step runs all its tasks at once, four lanes
//      per task. Every reflector is applied to the first four rows of Z and
//      logged (v, tau, p0); two consecutive time steps form one segment of
//      commuting reflectors (disjoint row windows). D, E of S and Z[0:4, :]
//      go to HBM.
//   2. k_eig: eigenvalues of S, one thread per eigenvalue index (all in
//      parallel): a multisection round on a grid of Sturm counts, bisection
//      until the eigenvalue is alone in its bracket, then Laguerre's
//      iteration toward it inside the bracket (about four steps);
//   3. eigenvectors of S: for an eigenvalue with no neighbour closer than
//      max(1e-6 ||S||, 1e-5 eV), a twisted factorisation of S - lambda I
//      (its pivots recomputed from sparse checkpoints instead of stored);
//      inside such a cluster, inverse iteration (tridiagonal LU with partial
//      pivoting, deterministic pseudo-random start) with the iterate made
//      orthogonal to the cluster's earlier members before every solve
//      (Peters & Wilkinson; the order of LAPACK's stein).
//      The eigenvector matrix U of S goes to HBM, the columns of the twisted
//      factorisations unnormalised, with their normalising factors apart;
//   4. Y[0:4, :] = Z[0:4, :] U, weights w_m = ||Y[0:4, m]||^2, Ritz values.
//
// k_rho (after the chemical potential is known): x = U (f(Lambda) Y[0:4,:]^T),
// then c = Z x by replaying the logged reflectors in reverse (segments in
// reverse order, the reflectors of one segment in parallel), and
// rho_{J,i} = V_J c for the rho row atoms J.
//
// Reflector convention: a logged (v1, v2, v3, tau, p0) is H = I - tau v v^T
// with v = (1, v1, v2, v3) on rows p0 .. p0+3; T <- H T H in order of the
// log, Z = H_1 H_2 ... H_n, so Z x applies H_n first.
#include <float.h>

#include "tb_internal.h"

namespace tbk {

constexpr int EIG_NT = 256;
constexpr int BAND_NT = 64;        // k_band: one wave per atom
constexpr int RHO_NT = 256;        // k_rho: four waves per atom
constexpr int RHO_REFW = 512;      // reflector-log window of k_rho (>= reflectors of any one segment)
constexpr int BW = 4;              // half-bandwidth of T
constexpr int SBR_NB = 8;          // stored lower diagonals of k_band (the fill reaches 7)
constexpr int SBR_LS = 9;          // LDS doubles per band column: concurrent tasks are 11 columns
                                   // apart, so a stride of 9 puts the 16 task groups of a wave on
                                   // 16 different bank pairs (a stride of 8 put them on 2)
constexpr int SBR_LAG = 3;         // time steps between the starts of consecutive sweeps

// Lane permutations within each quad of lanes (DPP quad_perm, no LDS round
// trip), for FP64 values: the value of lane (l & ~3) + P_j, P = (P0, P1, P2,
// P3) for the four lanes of the quad.
template <int PERM>
__device__ __forceinline__ double quad_perm_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), PERM, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), PERM, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int QP_XOR1 = 0xB1;    // (1, 0, 3, 2)
constexpr int QP_XOR2 = 0x4E;    // (2, 3, 0, 1)
template <int C> constexpr int QP_BCAST = C * 0x55;   // (C, C, C, C)

// Row m of the 4-column vectors in k_rho's LDS. The reflectors a replay step
// applies at once start 11 rows apart; with this skew their 16 leading rows
// in a wave fall on 16 different bank pairs (with a plain stride of 4
// doubles, on 4).
__host__ __device__ inline int xrow(int m) { return 4 * m + (m >> 3); }

// Columns of k_band's band storage: the matrix's plus the rows and columns a
// window at the end may reach (zero, and they stay zero).
__host__ __device__ inline int band_cols(int dmax) { return dmax + 8; }

// Reflectors of the reduction of a d x d T: sweep j (j = 0 .. d-3) has
// floor((d - 3 - j) / 4) + 1 tasks; replay segments: two time steps each.
int64_t band_reflectors(int d) {
  int64_t n = 0;
  for (int j = 0; j + 3 <= d; ++j) n += (d - 3 - j) / 4 + 1;
  return n > 0 ? n : 1;
}
int band_segments(int d) { return d >= 3 ? (3 * (d - 3) + 1 + 1) / 2 + 1 : 1; }

__device__ __forceinline__ double t_entry(const double* tab, int row, int col) {
  // lower triangle (row >= col) of the block tridiagonal T
  const int kr = row >> 2, ar = row & 3, kc = col >> 2, ac = col & 3;
  if (kr == kc) return tab[(size_t)kc * 32 + ar * 4 + ac];
  if (kr == kc + 1) return (ar <= ac) ? tab[(size_t)kc * 32 + 16 + ar * 4 + ac] : 0.0;
  return 0.0;
}

// Number of eigenvalues of the tridiagonal (D, E^2) below sigma: the number
// of sign changes in the sequence of leading principal minors of S - sigma I
// (Sturm), p_k = (D_k - sigma) p_{k-1} - E_{k-1}^2 p_{k-2}, p_{-1} = 1,
// p_{-2} = 0 -- equivalently the count of negative pivots of its LDL^T. The
// recurrence needs no division (the pivot form spends most of its issue slots
// on the FP64 reciprocal); p is brought back near 1 by a power of two every
// four steps, scaled by the larger of the last two (four steps change |p| by
// far less than the exponent range), and an exact zero becomes -2^-100 times
// its predecessor: a sign change, like the pivot form's -pivmin, and the next
// minor, ~ -E^2 p_{k-2}, keeps its size. E2s holds E^2 shifted by one (E2s[k] = E[k-1]^2,
// E2s[0] = 0) and d is a multiple of 4, so four steps take two 16-byte loads
// of each array.
__device__ __forceinline__ int sturm_count(const double* D, const double* E2s, int d, double sigma,
                                           double pivmin) {
  (void)pivmin;
  double p1 = 1.0, p2 = 0.0;
  int cnt = 0;
  for (int k = 0; k < d; k += 4) {
    const double2 d01 = *(const double2*)(D + k), d23 = *(const double2*)(D + k + 2);
    const double2 e01 = *(const double2*)(E2s + k), e23 = *(const double2*)(E2s + k + 2);
    const double dv[4] = {d01.x, d01.y, d23.x, d23.y}, ev[4] = {e01.x, e01.y, e23.x, e23.y};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double p = fma(dv[u] - sigma, p1, -(ev[u] * p2));
      if (p == 0.0) p = -0x1p-100 * p1;          // a sign change, like a pivot of -0
      cnt += (int)(((unsigned)__double2hiint(p) ^ (unsigned)__double2hiint(p1)) >> 31);
      p2 = p1;
      p1 = p;
    }
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1), fabs(p2)));
    p1 = __builtin_amdgcn_ldexp(p1, -e);
    p2 = __builtin_amdgcn_ldexp(p2, -e);
  }
  return cnt;
}

// The same count without the zero guard, for the common case: it only
// records whether some minor came out exactly zero (zero = true), and then
// the caller repeats the count with the guard. Without a zero the two
// recurrences are the same operations, so the counts agree bit for bit; the
// guard costs a multiply and two selects per row, about a quarter of a step.
__device__ __forceinline__ int sturm_count_nz(const double* D, const double* E2s, int d, double sigma, bool& zero) {
  double p1 = 1.0, p2 = 0.0;
  int cnt = 0;
  bool z = false;
  for (int k = 0; k < d; k += 4) {
    const double2 d01 = *(const double2*)(D + k), d23 = *(const double2*)(D + k + 2);
    const double2 e01 = *(const double2*)(E2s + k), e23 = *(const double2*)(E2s + k + 2);
    const double dv[4] = {d01.x, d01.y, d23.x, d23.y}, ev[4] = {e01.x, e01.y, e23.x, e23.y};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double p = fma(dv[u] - sigma, p1, -(ev[u] * p2));
      z |= (p == 0.0);
      cnt += (int)(((unsigned)__double2hiint(p) ^ (unsigned)__double2hiint(p1)) >> 31);
      p2 = p1;
      p1 = p;
    }
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1), fabs(p2)));
    p1 = __builtin_amdgcn_ldexp(p1, -e);
    p2 = __builtin_amdgcn_ldexp(p2, -e);
  }
  zero = z;
  return cnt;
}

// The count at sigma: the unguarded recurrence, repeated with the guard in
// the rare case of an exact zero minor.
__device__ __forceinline__ int sturm_count_fast(const double* D, const double* E2s, int d, double sigma,
                                                double pivmin) {
  bool zero;
  const int c = sturm_count_nz(D, E2s, d, sigma, zero);
  return zero ? sturm_count(D, E2s, d, sigma, pivmin) : c;
}

// Sturm count at sigma (as sturm_count_nz) together with the ratios
// g1 = p'/p and g2 = p''/p of the characteristic polynomial p(x) = det(S - x I)
// at x = sigma: the minors recurrence differentiated once and twice,
//   p'_k  = (D_k - x) p'_{k-1}  - p_{k-1}      - E_{k-1}^2 p'_{k-2},
//   p''_k = (D_k - x) p''_{k-1} - 2 p'_{k-1}   - E_{k-1}^2 p''_{k-2},
// rescaled together with p (the ratios are unchanged). zero: some minor came
// out exactly zero (the count is then repeated with the guard).
__device__ __forceinline__ int sturm_lag(const double* D, const double* E2s, int d, double sigma, double& g1,
                                         double& g2, bool& zero) {
  double p1 = 1.0, p2 = 0.0, q1 = 0.0, q2 = 0.0, s1 = 0.0, s2 = 0.0;
  int cnt = 0;
  bool z = false;
  for (int k = 0; k < d; k += 4) {
    const double2 d01 = *(const double2*)(D + k), d23 = *(const double2*)(D + k + 2);
    const double2 e01 = *(const double2*)(E2s + k), e23 = *(const double2*)(E2s + k + 2);
    const double dv[4] = {d01.x, d01.y, d23.x, d23.y}, ev[4] = {e01.x, e01.y, e23.x, e23.y};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double a = dv[u] - sigma;
      const double p = fma(a, p1, -(ev[u] * p2));
      const double q = fma(a, q1, -fma(ev[u], q2, p1));
      const double r = fma(a, s1, -fma(ev[u], s2, 2.0 * q1));
      z |= (p == 0.0);
      cnt += (int)(((unsigned)__double2hiint(p) ^ (unsigned)__double2hiint(p1)) >> 31);
      p2 = p1; p1 = p;
      q2 = q1; q1 = q;
      s2 = s1; s1 = r;
    }
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(p1), fabs(p2)));
    p1 = __builtin_amdgcn_ldexp(p1, -e); p2 = __builtin_amdgcn_ldexp(p2, -e);
    q1 = __builtin_amdgcn_ldexp(q1, -e); q2 = __builtin_amdgcn_ldexp(q2, -e);
    s1 = __builtin_amdgcn_ldexp(s1, -e); s2 = __builtin_amdgcn_ldexp(s2, -e);
  }
  zero = z;
  g1 = q1 / p1;
  g2 = s1 / p1;
  return cnt;
}

// Eigenvalue t of the tridiagonal S of n rows (D and the shifted squares E2s
// as for sturm_count) from a bracket [l, h] whose Sturm counts are
// cl <= t < ch. Bisection narrows the bracket until it holds
// eigenvalue t alone (cl == t, ch == t + 1); then Laguerre's iteration for the
// real-rooted polynomial p of degree n: with G = p'/p and H = G^2 - p''/p the
// two iterates x - n / (G +- sqrt((n - 1)(n H - G^2))) lie on either side of x,
// each between x and the nearest root on its side, and converge cubically to
// it. The Sturm count at x says on which side eigenvalue t lies (the bracket
// holds no other), so the step goes that way; every count also narrows the
// bracket, and a step that would leave it (rounding) becomes the midpoint.
// Stops when a step is below 1e-12 anorm (the next error is then at rounding
// level) or the bracket is below 4 eps max(|l|, |h|) + pivmin.
__device__ double eig_laguerre(const double* D, const double* E2s, int n, int t, double l, double h, int cl,
                               int ch, double anorm, double pivmin) {
  const double nd = (double)n;
  auto narrow = [&](double x, int c) {
    if (c <= t) { l = x; cl = c; } else { h = x; ch = c; }
  };
  auto done = [&]() { return h - l <= 4.0 * DBL_EPSILON * fmax(fabs(l), fabs(h)) + pivmin; };
  int it = 0;
  while (!(cl == t && ch == t + 1) && !done() && it < 128) {
    const double m = 0.5 * (l + h);
    narrow(m, sturm_count_fast(D, E2s, n, m, pivmin));
    ++it;
  }
  double x = 0.5 * (l + h);
  while (!done() && it < 128) {
    ++it;
    double g1, g2;
    bool zero;
    int c = sturm_lag(D, E2s, n, x, g1, g2, zero);
    if (zero) c = sturm_count(D, E2s, n, x, pivmin);
    narrow(x, c);
    if (!(isfinite(g1) && isfinite(g2))) {        // x is an eigenvalue to rounding
      if (c == t + 1 || c == t) return x;
      x = 0.5 * (l + h);
      continue;
    }
    const double hh = g1 * g1 - g2;
    const double disc = sqrt(fmax((nd - 1.0) * (nd * hh - g1 * g1), 0.0));
    const double den = (c > t) ? g1 + disc : g1 - disc;     // c > t: eigenvalue t lies left of x
    const double step = nd / den;
    const double xn = x - step;
    if (fabs(step) <= 1e-12 * anorm) return fmin(fmax(xn, l), h);
    x = (xn > l && xn < h) ? xn : 0.5 * (l + h);
  }
  return 0.5 * (l + h);
}

// 1 / q from the hardware reciprocal refined by one Newton step (relative
// error near the unit roundoff).
__device__ __forceinline__ double rcp_nr(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

// Deterministic start vector component for eigenvalue t, row k: uniform in
// (-1, 1) from an integer hash. Signs alone (+-1) are not enough: a
// mirror-symmetric block of S has eigenvectors that are exactly orthogonal to
// every symmetric +-1 pattern.
__device__ __forceinline__ double start_val(int t, int k) {
  unsigned int h = (unsigned int)k * 2654435761u ^ ((unsigned int)t * 40503u + 0x9e3779b9u);
  h ^= h >> 15; h *= 0x2c1b3c6du; h ^= h >> 12; h *= 0x297a2d39u; h ^= h >> 15;
  return ((double)(h >> 8) + 0.5) * (2.0 / 16777216.0) - 1.0;
}

// (S - lam I) x = small * b by LU with partial pivoting; b from start_val
// (bcol == nullptr) or from the column bcol (stride ld). x is written to xcol
// (stride ld; may alias bcol). The right-hand side is scaled by the pivot
// floor so that a near-singular last pivot gives |x| of order one rather than
// 1/eps. Scratch: 4 values per row at scr[(k * 4 + f) * ns] (coalesced
// over the workgroup). UT: element type of the columns of U (double, or
// float after the FP32 recursion). Returns ||x||^2 of the computed x (before
// its rounding to UT).
template <typename UT>
__device__ double inv_solve(const double* D, const double* E, int d, double lam, double small, int t,
                            const UT* bcol, UT* xcol, size_t ld, double* scr, int ns) {
  double cd = D[0] - lam;
  double cu = d > 1 ? E[0] : 0.0;
  double cb = small * (bcol ? bcol[0] : start_val(t, 0));
  for (int k = 0; k + 1 < d; ++k) {
    const double sub = E[k];
    const double nd = D[k + 1] - lam;
    const double nu = (k + 2 < d) ? E[k + 1] : 0.0;
    const double nb = small * (bcol ? bcol[(size_t)(k + 1) * ld] : start_val(t, k + 1));
    double* sk = scr + (size_t)k * 4 * ns;
    if (fabs(cd) >= fabs(sub)) {
      const double piv = (cd != 0.0) ? cd : small;
      const double l = sub / piv;
      sk[0] = piv; sk[ns] = cu; sk[2 * ns] = 0.0; sk[3 * ns] = cb;
      cd = nd - l * cu; cu = nu; cb = nb - l * cb;
    } else {
      const double l = cd / sub;
      sk[0] = sub; sk[ns] = nd; sk[2 * ns] = nu; sk[3 * ns] = nb;
      cd = cu - l * nd; cu = -l * nu; cb = cb - l * nb;
    }
  }
  double* sl = scr + (size_t)(d - 1) * 4 * ns;
  sl[0] = cd; sl[ns] = 0.0; sl[2 * ns] = 0.0; sl[3 * ns] = cb;
  double x1 = 0.0, x2 = 0.0, nrm = 0.0;
  for (int k = d - 1; k >= 0; --k) {
    const double* sk = scr + (size_t)k * 4 * ns;
    double piv = sk[0];
    if (fabs(piv) < small) piv = (piv < 0.0) ? -small : small;
    const double x = (sk[3 * ns] - sk[ns] * x1 - sk[2 * ns] * x2) / piv;
    xcol[(size_t)k * ld] = (UT)x;
    nrm += x * x;
    x2 = x1; x1 = x;
  }
  return nrm;
}

// Eigenvector of a cluster member t at position pos > 0 of its cluster, or of
// the first member (pos = 0), by inverse iteration in the order of Peters &
// Wilkinson and LAPACK's stein: the iterate is made orthogonal to the
// earlier members (the pos columns before xc, cs elements apart, already
// normalised) before every solve, so that each solve amplifies the
// directions of the cluster's invariant subspace those members do not cover.
// (Orthogonalising only after the solves fails on an exactly degenerate
// eigenvalue: the solves converge into the earlier members' span and the
// Gram-Schmidt remainder is rounding noise.) Two solves for the first member,
// three for the others; when orthogonalisation removes most of an iterate,
// the member starts again from another pseudo-random vector. The result in
// xc (stride ld) is normalised.
template <typename UT>
__device__ void cluster_vector(const double* D, const double* E, int d, double lam, double small, int t, int pos,
                               UT* xc, size_t ld, size_t cs, double* scr, int ns) {
  auto orth = [&]() {
    for (int rep = 0; rep < 2; ++rep) {
      for (int p = 1; p <= pos; ++p) {
        const UT* uj = xc - (size_t)p * cs;
        double dot = 0.0;
        for (int k = 0; k < d; ++k) dot += (double)uj[(size_t)k * ld] * (double)xc[(size_t)k * ld];
        for (int k = 0; k < d; ++k)
          xc[(size_t)k * ld] = (UT)((double)xc[(size_t)k * ld] - dot * (double)uj[(size_t)k * ld]);
      }
    }
    double nrm = 0.0;
    for (int k = 0; k < d; ++k) nrm += (double)xc[(size_t)k * ld] * (double)xc[(size_t)k * ld];
    return nrm;
  };
  auto scale = [&](double nrm) {
    const double sc = 1.0 / sqrt(nrm);
    for (int k = 0; k < d; ++k) xc[(size_t)k * ld] = (UT)((double)xc[(size_t)k * ld] * sc);
  };
  int seed = t;
  for (int attempt = 0; attempt < 4; ++attempt) {
    for (int k = 0; k < d; ++k) xc[(size_t)k * ld] = (UT)start_val(seed, k);
    scale(pos > 0 ? orth() : (double)d);
    bool ok = true;
    for (int s = 0; s < (pos > 0 ? 3 : 2); ++s) {
      scale(inv_solve<UT>(D, E, d, lam, small, t, xc, xc, ld, scr, ns));
      if (pos > 0) {
        const double nrm = orth();
        if (!(nrm > 0.25)) { ok = false; scale(nrm > 0.0 ? nrm : 1.0); break; }
        scale(nrm);
      }
    }
    if (ok) return;
    seed += 7919 * (attempt + 1) + d;
  }
}

// Eigenvector of the tridiagonal (D, E; E2 = E^2) for an eigenvalue lam that
// is not in a cluster, by a twisted factorisation of S - lam I (Godunov;
// Fernando; Parlett & Dhillon): forward pivots d+_k of L D L^T, backward
// pivots d-_k of U D U^T, the twist index r where
// |gamma_r| = |d+_r + d-_r - (D_r - lam)| is smallest, then z_r = 1 and
// z_k = -E_k z_{k+1} / d+_k (k < r), z_k = -E_{k-1} z_{k-1} / d-_k (k > r).
// Pivots of magnitude below `small` are replaced by +-small. The vector goes
// to xcol (stride ld) unnormalised; the return value is the factor that
// normalises it (applied by the readers). ACC: also accumulates
// y[c] = sum_k R1[c d + k] z_k, the column's projection on the first four rows
// of Z (R1 in LDS, row stride d), as z is produced.
// The pivots are not stored: every CK-th forward pivot
// d+_k and backward pivot d-_k (k a multiple of CK) goes to the thread's
// checkpoint scratch (ck[j * ns], 2 ceil(d / CK) values), and each pass that
// needs a run of pivots in the other order recomputes the run from its
// checkpoint into registers with the same operations (explicit FMAs), so the
// values agree bit for bit with the first computation. Passes: forward pivots;
// backward pivots with the forward ones of each run recomputed, giving the
// twist index; z_k for k < r (forward pivots recomputed per run, consumed in
// reverse); z_k for k > r (backward pivots recomputed per run from the next
// run's checkpoint, consumed in order).
template <bool ACC, typename UT>
__device__ double twisted_ck(const double* D, const double* E, const double* E2, int d, double lam, double small,
                             UT* xcol, size_t ld, double* ck, int ns, const double* R1 = nullptr,
                             double* y = nullptr) {
  constexpr int CK = 8;
  const int nck = (d + CK - 1) / CK;
  double* ckf = ck;                              // d+ at rows c CK
  double* ckb = ck + (size_t)nck * ns;           // d- at rows c CK
  auto guard = [&](double v) { return fabs(v) < small ? (v < 0.0 ? -small : small) : v; };
  auto fwd = [&](double q, int k) { return guard(fma(-E2[k - 1], rcp_nr(q), D[k] - lam)); };   // d+_k
  auto bwd = [&](double m, int k) { return guard(fma(-E2[k], rcp_nr(m), D[k] - lam)); };       // d-_k
  double q = guard(D[0] - lam);
  ckf[0] = q;
  for (int k = 1; k < d; ++k) {
    q = fwd(q, k);
    if ((k & (CK - 1)) == 0) ckf[(size_t)(k / CK) * ns] = q;
  }
  int r = d - 1;
  double best = 3.0e300, m = 0.0;
  // each sweep over the runs loads the next run's checkpoint while the
  // current run is recomputed (the load is off the recurrence's chain)
  double ckn = ckf[(size_t)(nck - 1) * ns];
  for (int c = nck - 1; c >= 0; --c) {
    const int k0 = c * CK;
    double pv[CK];
    pv[0] = ckn;
    if (c > 0) ckn = ckf[(size_t)(c - 1) * ns];
#pragma unroll
    for (int u = 1; u < CK; ++u) pv[u] = (k0 + u < d) ? fwd(pv[u - 1], k0 + u) : 0.0;
#pragma unroll
    for (int u = CK - 1; u >= 0; --u) {
      const int k = k0 + u;
      if (k >= d) continue;
      double gam;
      if (k == d - 1) {
        m = guard(D[k] - lam);
        gam = fabs(pv[u]);                       // gamma_{d-1} = d+_{d-1}
      } else {
        m = bwd(m, k);
        gam = fabs(pv[u] + m - (D[k] - lam));
      }
      if (gam < best) { best = gam; r = k; }
    }
    ckb[(size_t)c * ns] = m;                     // d-_{k0}
  }
  double z = 1.0, nrm = 1.0;
  xcol[(size_t)r * ld] = (UT)1.0;
  double y0 = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0;
  if constexpr (ACC) { y0 = R1[r]; y1 = R1[(size_t)d + r]; y2 = R1[(size_t)2 * d + r]; y3 = R1[(size_t)3 * d + r]; }
  auto acc = [&](int k, double zk) {
    xcol[(size_t)k * ld] = (UT)zk;
    nrm += zk * zk;
    if constexpr (ACC) {
      y0 += R1[k] * zk; y1 += R1[(size_t)d + k] * zk; y2 += R1[(size_t)2 * d + k] * zk; y3 += R1[(size_t)3 * d + k] * zk;
    }
  };
  // k < r: z_k = -E_k z_{k+1} / d+_k
  ckn = ckf[(size_t)((r - 1) / CK) * ns];
  for (int c = (r - 1) / CK; r > 0 && c >= 0; --c) {
    const int k0 = c * CK;
    double pv[CK];
    pv[0] = ckn;
    if (c > 0) ckn = ckf[(size_t)(c - 1) * ns];
#pragma unroll
    for (int u = 1; u < CK; ++u) pv[u] = (k0 + u < d) ? fwd(pv[u - 1], k0 + u) : 1.0;
#pragma unroll
    for (int u = CK - 1; u >= 0; --u) {
      const int k = k0 + u;
      if (k >= r) continue;
      z = -E[k] * z * rcp_nr(pv[u]);
      acc(k, z);
    }
  }
  // k > r: z_k = -E_{k-1} z_{k-1} / d-_k
  z = 1.0;
  ckn = ((r + 1) / CK + 1 < nck) ? ckb[(size_t)((r + 1) / CK + 1) * ns] : 0.0;
  for (int c = (r + 1) / CK; c < nck; ++c) {
    const int k0 = c * CK;
    double mv[CK];
    // d- over the run, downward from the next run's checkpoint (or from row d - 1)
    double mm = ckn;
    ckn = (c + 2 < nck) ? ckb[(size_t)(c + 2) * ns] : 0.0;
#pragma unroll
    for (int u = CK - 1; u >= 0; --u) {
      const int k = k0 + u;
      if (k >= d) { mv[u] = 1.0; continue; }
      mm = (k == d - 1) ? guard(D[k] - lam) : bwd(mm, k);
      mv[u] = mm;
    }
#pragma unroll
    for (int u = 0; u < CK; ++u) {
      const int k = k0 + u;
      if (k <= r || k >= d) continue;
      z = -E[k - 1] * z * rcp_nr(mv[u]);
      acc(k, z);
    }
  }
  if constexpr (ACC) { y[0] = y0; y[1] = y1; y[2] = y2; y[3] = y3; }
  return 1.0 / sqrt(nrm);
}

// Band -> tridiagonal reduction, one wave per atom. LDS: the lower band
// L[c * SBR_LS + t] = A[c + t][c] (t < SBR_NB) over band_cols(dmax) columns,
// then the first four rows of Z (row stride zs, odd). At time step t the
// active sweeps are j in [jmin, jmax] with task s = t - 3 j and window p0 =
// 4 t + 1 - 11 j <= d - 2; lanes 4 g .. 4 g + 3 take task jmax - g (then -16,
// -32 ... while tasks remain). Each of the four lanes of a task forms the
// reflector from the column it annihilates, then lane q transforms: the
// column p0 - 3 + q left of the window (q < 3, tasks after the first of a
// sweep), row q of the symmetric 4x4 window block (rank-2 form
// A <- A - v w^T - w v^T, w = p - (tau/2)(p.v) v, p = tau A v; the four p_q
// summed over the quad by DPP permutes), row p0 + 4 + q below the window, and
// row q of Z. Every lane loads everything it needs before any store, and the
// LDS operations of a wave complete in issue order; wave-scope fences order
// the time steps.
__global__ void __launch_bounds__(BAND_NT) k_band(EigArgs g) {
  extern __shared__ double bsm[];
  const int lane = threadIdx.x;
  const int atom = g.atom0 + blockIdx.x;
  if (atom >= g.n_atoms) return;
  const int dmax = 4 * g.r_max;
  const int nc = band_cols(dmax);
  const int zs = nc | 1;                             // Z row stride (odd: rows on different banks)
  double* L = bsm;                                   // [nc][SBR_LS]
  double* Zr = bsm + (size_t)nc * SBR_LS;            // [4][zs]
  const int d = 4 * g.kused[atom];
  const double* tab = g.tab + (size_t)atom * g.r_max * 32;
  for (int q = lane; q < nc * SBR_LS; q += BAND_NT) {
    const int c = q / SBR_LS, t = q % SBR_LS;
    L[q] = (t <= BW && c + t < d) ? t_entry(tab, c + t, c) : 0.0;
  }
  for (int q = lane; q < 4 * zs; q += BAND_NT) Zr[q] = (q % zs == q / zs) ? 1.0 : 0.0;
  auto wave_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  wave_sync();
  double* lv = g.ref_v + (size_t)atom * g.ref_max * 4;
  uint16_t* lp = g.ref_p + (size_t)atom * g.ref_max;
  int* seg = g.seg + (size_t)atom * g.seg_max;
  const int grp = lane >> 2, q = lane & 3;
  int64_t nref = 0;
  int nseg = 0;
  const int T = d >= 3 ? SBR_LAG * (d - 3) + 1 : 0;
  for (int t = 0; t < T; ++t) {
    if ((t & 1) == 0) {                             // a segment: time steps t, t + 1
      if (lane == 0 && nseg < g.seg_max) seg[nseg] = (int)nref;
      ++nseg;
    }
    const int jmax = min(t / SBR_LAG, d - 3);
    const int num = 4 * t + 3 - d;
    const int jmin = num > 0 ? (num + 10) / 11 : 0;
    const int ntask = jmax - jmin + 1;
    for (int b0 = 0; b0 < ntask; b0 += 16) {
      const int ti = b0 + grp;
      if (ti < ntask) {
        const int j = jmax - ti, s = t - SBR_LAG * j;
        const int p0 = 4 * t + 1 - 11 * j;          // = j + 1 + 4 s
        const int col = s == 0 ? j : p0 - 4;        // the column annihilated
        const double* Lc = L + (size_t)col * SBR_LS + (p0 - col);
        const double x0 = Lc[0], x1 = Lc[1], x2 = Lc[2], x3 = Lc[3];
        // reflector H = I - tau v v^T, v = (1, v1, v2, v3), H x = (beta, 0, 0, 0)
        const double sig = x1 * x1 + x2 * x2 + x3 * x3;
        double v1 = 0.0, v2 = 0.0, v3 = 0.0, tau = 0.0, beta = x0;
        if (sig != 0.0) {
          // |x| and 1/|x| from the hardware reciprocal square root, each
          // refined by one Newton step; tau = (beta - x0) / beta = 1 + |x0| / |x|
          const double s2 = fma(x0, x0, sig);
          double rs = __builtin_amdgcn_rsq(s2);
          rs = rs * fma(-0.5 * s2 * rs, rs, 1.5);
          double mu = s2 * rs;
          mu = fma(fma(-mu, mu, s2), 0.5 * rs, mu);
          beta = x0 >= 0.0 ? -mu : mu;
          const double iv0 = rcp_nr(x0 - beta);
          v1 = x1 * iv0; v2 = x2 * iv0; v3 = x3 * iv0;
          tau = fma(fabs(x0), rs, 1.0);
        }
        const double vv[4] = {1.0, v1, v2, v3};
        const double vq = vv[q];
        // loads: left column, window row q, row below, Z row
        const bool left = s > 0 && q < 3;
        const int cl = p0 - 3 + q;
        double ya[4], yd[4], yr[4], yz[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ya[i] = left ? L[(size_t)cl * SBR_LS + (p0 + i - cl)] : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
          yd[m] = m <= q ? L[(size_t)(p0 + m) * SBR_LS + (q - m)] : L[(size_t)(p0 + q) * SBR_LS + (m - q)];
#pragma unroll
        for (int m = 0; m < 4; ++m) yr[m] = L[(size_t)(p0 + m) * SBR_LS + (4 + q - m)];
#pragma unroll
        for (int m = 0; m < 4; ++m) yz[m] = Zr[(size_t)q * zs + p0 + m];
        // left column and row below and Z row: y <- H y
        const double da = ya[0] + v1 * ya[1] + v2 * ya[2] + v3 * ya[3];
        const double dr = yr[0] + v1 * yr[1] + v2 * yr[2] + v3 * yr[3];
        const double dz = yz[0] + v1 * yz[1] + v2 * yz[2] + v3 * yz[3];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ya[i] -= tau * da * vv[i];
          yr[i] -= tau * dr * vv[i];
          yz[i] -= tau * dz * vv[i];
        }
        // window block: p_q = tau (A v)_q, K = (tau/2) sum p v, w = p - K v
        const double pq = tau * (yd[0] + v1 * yd[1] + v2 * yd[2] + v3 * yd[3]);
        double kq = pq * vq;
        kq += quad_perm_d<QP_XOR1>(kq);
        kq += quad_perm_d<QP_XOR2>(kq);
        const double wq = pq - 0.5 * tau * kq * vq;
        double wm[4];
        wm[0] = quad_perm_d<QP_BCAST<0>>(wq); wm[1] = quad_perm_d<QP_BCAST<1>>(wq);
        wm[2] = quad_perm_d<QP_BCAST<2>>(wq); wm[3] = quad_perm_d<QP_BCAST<3>>(wq);
#pragma unroll
        for (int m = 0; m < 4; ++m) yd[m] -= vq * wm[m] + wq * vv[m];
        // stores
        L[(size_t)col * SBR_LS + (p0 + q - col)] = q == 0 ? beta : 0.0;
        if (left) {
#pragma unroll
          for (int i = 0; i < 4; ++i) L[(size_t)cl * SBR_LS + (p0 + i - cl)] = ya[i];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if (m <= q) L[(size_t)(p0 + m) * SBR_LS + (q - m)] = yd[m];
#pragma unroll
        for (int m = 0; m < 4; ++m) L[(size_t)(p0 + m) * SBR_LS + (4 + q - m)] = yr[m];
#pragma unroll
        for (int m = 0; m < 4; ++m) Zr[(size_t)q * zs + p0 + m] = yz[m];
        const int64_t slot = nref + ti;
        if (q == 0 && slot < g.ref_max) {
          *(double4*)(lv + 4 * slot) = make_double4(v1, v2, v3, tau);
          lp[slot] = (uint16_t)p0;
        }
      }
    }
    nref += ntask > 0 ? ntask : 0;
    wave_sync();
  }
  if (lane == 0) {
    g.ref_n[atom] = (int)(nref < g.ref_max ? nref : g.ref_max);
    const int ns = nseg < g.seg_max ? nseg : g.seg_max;
    g.seg_n[2 * atom] = ns;
    g.seg_n[2 * atom + 1] = ns;
    if (nseg > g.seg_max) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_SEG_OVERFLOW);
    if (nref > g.ref_max) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_REFLOG_OVERFLOW);
  }
  // tridiagonal S (D, E) and Z[0:4, :]
  double* tri = g.tri + (size_t)atom * 2 * dmax;
  double* r1 = g.y1 + (size_t)atom * 4 * dmax;
  for (int k = lane; k < d; k += BAND_NT) {
    tri[k] = L[(size_t)k * SBR_LS];
    tri[dmax + k] = (k + 1 < d) ? L[(size_t)k * SBR_LS + 1] : 0.0;
  }
  for (int qq = lane; qq < 4 * d; qq += BAND_NT) {
    const int c = qq / d, m = qq % d;
    r1[(size_t)c * dmax + m] = Zr[(size_t)c * zs + m];
  }
}

template <typename UT>
__global__ void __launch_bounds__(EIG_NT, 4) k_eig(EigArgs g) {
  extern __shared__ double esm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = blockDim.x, nw = nt / 64;        // threads: 64 ceil(4 r_max / 64), at most EIG_NT
  const int dmax = 4 * g.r_max;
  double* R1 = esm;                        // [4][d] first rows of Z
  double* Dg = R1 + (size_t)4 * dmax;      // [dmax] diagonal of S
  double* Eg = Dg + dmax;                  // [dmax] off-diagonal of S (E[k]: k, k+1)
  double* E2 = Eg + dmax;                  // [dmax] E^2
  double* lam_s = E2 + dmax;               // [dmax] eigenvalues (ascending)
  double* E2s = lam_s + dmax;              // [dmax] E^2 shifted by one (E2s[k] = E[k-1]^2)
  double* red = E2s + dmax;                // [EIG_NT/64][4]
  int* pos_s = (int*)(red + 4 * (EIG_NT / 64));   // [dmax] position inside a cluster
  __shared__ int s_atom, s_maxpos;
  __shared__ double s_lo, s_hi, s_e2max;
  double* scr = g.scratch + (size_t)blockIdx.x * dmax * 4 * nt + tid;

  for (;;) {
    if (tid == 0) s_atom = atomicAdd(g.counter, 1);
    __syncthreads();
    const int atom = g.atom0 + s_atom;
    if (atom >= g.n_atoms) break;
    const int K = g.kused[atom];
    const int d = 4 * K;
    const double* tri = g.tri + (size_t)atom * 2 * dmax;
    const double* r1 = g.y1 + (size_t)atom * 4 * dmax;
    for (int q = tid; q < 4 * d; q += nt) {
      const int c = q / d, m = q % d;
      R1[q] = r1[(size_t)c * dmax + m];
    }

    // ---- 2. tridiagonal S, Gershgorin interval, eigenvalues (multisection
    // round, then bisection and Laguerre's iteration per eigenvalue)
    double glo = 1e300, ghi = -1e300, e2m = 0.0;
    for (int k = tid; k < d; k += nt) {
      const double Dk = tri[k];
      const double Ek = (k + 1 < d) ? tri[dmax + k] : 0.0;
      const double Em = (k > 0) ? tri[dmax + k - 1] : 0.0;
      Dg[k] = Dk; Eg[k] = Ek; E2[k] = Ek * Ek; E2s[k] = Em * Em;
      const double rad = fabs(Ek) + fabs(Em);
      glo = fmin(glo, Dk - rad); ghi = fmax(ghi, Dk + rad); e2m = fmax(e2m, Ek * Ek);
    }
    for (int off = 32; off > 0; off >>= 1) {
      glo = fmin(glo, __shfl_xor(glo, off, 64));
      ghi = fmax(ghi, __shfl_xor(ghi, off, 64));
      e2m = fmax(e2m, __shfl_xor(e2m, off, 64));
    }
    if (lane == 0) { red[wave * 4] = glo; red[wave * 4 + 1] = ghi; red[wave * 4 + 2] = e2m; }
    __syncthreads();
    if (tid == 0) {
      double a = 1e300, b = -1e300, e = 0.0;
      for (int w = 0; w < nw; ++w) { a = fmin(a, red[w * 4]); b = fmax(b, red[w * 4 + 1]); e = fmax(e, red[w * 4 + 2]); }
      const double pad = 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + 1e-300;
      s_lo = a - pad; s_hi = b + pad; s_e2max = e;
    }
    __syncthreads();
    const double lo0 = s_lo, hi0 = s_hi;
    const double anorm = fmax(fabs(lo0), fabs(hi0));
    const double pivmin = DBL_MIN * fmax(1.0, s_e2max);
    // one multisection round on a grid of nt points (one Sturm count per
    // thread), then each eigenvalue is bisected from its grid cell
    int* cnt_s = pos_s + dmax;                     // [nt]
    const double hg = (hi0 - lo0) / (nt + 1);
    cnt_s[tid] = sturm_count_fast(Dg, E2s, d, lo0 + (tid + 1) * hg, pivmin);
    __syncthreads();
    for (int t = tid; t < d; t += nt) {
      // cells with count(left) <= t < count(right); the ends count 0 and d
      int il = -1, ih = nt;
      while (ih - il > 1) {
        const int im = (il + ih) >> 1;
        if (cnt_s[im] <= t) il = im; else ih = im;
      }
      const double l = il < 0 ? lo0 : lo0 + (il + 1) * hg, h = ih >= nt ? hi0 : lo0 + (ih + 1) * hg;
      lam_s[t] = eig_laguerre(Dg, E2s, d, t, l, h, il < 0 ? 0 : cnt_s[il], ih >= nt ? d : cnt_s[ih], anorm, pivmin);
    }
    __syncthreads();
    // ---- 3. clusters and inverse iteration
    const double ctol = fmax(1e-6 * anorm, 1e-5);
    const double small = DBL_EPSILON * anorm + 1e-300;
    int mp = 0;
    for (int t = tid; t < d; t += nt) {
      int p = 0;
      while (t - p - 1 >= 0 && lam_s[t - p] - lam_s[t - p - 1] < ctol) ++p;
      pos_s[t] = p;
      mp = p > mp ? p : mp;
    }
    for (int off = 32; off > 0; off >>= 1) { const int o = __shfl_xor(mp, off, 64); mp = o > mp ? o : mp; }
    if (tid == 0) s_maxpos = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&s_maxpos, mp);
    __syncthreads();
    const int maxpos = s_maxpos;
    UT* Ua = (UT*)g.evec + (size_t)atom * dmax * dmax;      // column t of U at Ua + t dmax
    double* vsc = g.vsc + (size_t)atom * dmax;              // normalising factor of column t
    for (int round = 0; round <= maxpos; ++round) {
      for (int t = tid; t < d; t += nt) {
        if (pos_s[t] != round) continue;
        UT* xc = Ua + (size_t)t * dmax;
        if (round == 0 && (t + 1 >= d || pos_s[t + 1] == 0)) {
          // not in a cluster: twisted factorisation (column scale kept apart),
          // which also forms Y[0:4, t] = Z[0:4, :] U[:, t]; the outputs of
          // the column are written here and skipped in step 4
          double ya[4];
          const double sc = twisted_ck<true, UT>(Dg, Eg, E2, d, lam_s[t], small, xc, 1, scr, nt, R1, ya);
          vsc[t] = sc;
          double* y1o = g.y1 + (size_t)atom * 4 * dmax;
          const double a0 = ya[0] * sc, a1 = ya[1] * sc, a2 = ya[2] * sc, a3 = ya[3] * sc;
          g.lam[(size_t)atom * dmax + t] = lam_s[t];
          g.wgt[(size_t)atom * dmax + t] = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
          y1o[t] = a0; y1o[dmax + t] = a1; y1o[2 * dmax + t] = a2; y1o[3 * dmax + t] = a3;
          continue;
        }
        vsc[t] = 1.0;                                // normalised here
        cluster_vector<UT>(Dg, Eg, d, lam_s[t], small, t, round, xc, 1, dmax, scr, nt);
      }
      __syncthreads();
    }
    // ---- 4. Y[0:4, t] = Z[0:4, :] U[:, t], weights, outputs
    double* lam = g.lam + (size_t)atom * dmax;
    double* wgt = g.wgt + (size_t)atom * dmax;
    double* y1 = g.y1 + (size_t)atom * 4 * dmax;
    for (int t = tid; t < dmax; t += nt) {
      if (t < d && pos_s[t] == 0 && (t + 1 >= d || pos_s[t + 1] == 0)) continue;   // written in step 3
      if (t < d) {
        const UT* xc = Ua + (size_t)t * dmax;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
        for (int k = 0; k < d; ++k) {
          const double x = (double)xc[k];
          a0 += R1[k] * x; a1 += R1[(size_t)d + k] * x; a2 += R1[(size_t)2 * d + k] * x; a3 += R1[(size_t)3 * d + k] * x;
        }
        const double sc = vsc[t];
        a0 *= sc; a1 *= sc; a2 *= sc; a3 *= sc;
        lam[t] = lam_s[t];
        wgt[t] = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
        y1[t] = a0; y1[dmax + t] = a1; y1[2 * dmax + t] = a2; y1[3 * dmax + t] = a3;
      } else {
        lam[t] = 0.0; wgt[t] = 0.0;
        y1[t] = 0.0; y1[dmax + t] = 0.0; y1[2 * dmax + t] = 0.0; y1[3 * dmax + t] = 0.0;
      }
    }
    if (tid == 0) atomicMax((unsigned long long*)&g.stats[ST_MAX_CLUSTER_POS], (unsigned long long)maxpos);
    __syncthreads();
  }
}

// Orbital seeds: T is the direct sum of four scalar chains, chain c on the
// rows 4k + c (k < K) of the block layout (A_k, B_k diagonal). Each chain is
// its own symmetric tridiagonal (D = alpha^c, E = beta^c) and is solved on
// its own, with no band reduction (Z = I, an empty rotation log): Laguerre
// on the chain's Sturm sequence, clusters only among the chain's own
// eigenvalues, eigenvectors by twisted factorisation or inverse iteration on
// the chain, written to the rows 4k + c of U (the other rows zero).
// Eigenpair t = c K + j is the j-th of chain c, and Y[0:4, t] = U[0:4, t] is
// nonzero in row c only. The chains are stored chain-major at a stride Kp =
// K rounded up to 4 (the Sturm count reads four rows at a time), padded with
// D = 1e30, E = 0: rows that add no sign change below any eigenvalue.
template <typename UT>
__global__ void __launch_bounds__(EIG_NT, 4) k_eig_chains(EigArgs g) {
  extern __shared__ double esm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = blockDim.x, nw = nt / 64;
  const int dmax = 4 * g.r_max;
  const int DP = 4 * ((g.r_max + 3) & ~3);
  double* Dg = esm;                        // [4][Kp] chain-major, padded
  double* Eg = Dg + DP;
  double* E2 = Eg + DP;
  double* E2s = E2 + DP;                   // E2s[k] = E[k-1]^2 within the chain
  double* lam_s = E2s + DP;                // [dmax] eigenvalues, ascending within each chain
  double* red = lam_s + dmax;              // [EIG_NT/64][4]
  int* pos_s = (int*)(red + 4 * (EIG_NT / 64));   // [dmax] position inside a cluster
  __shared__ int s_atom, s_maxpos;
  __shared__ double s_lo, s_hi, s_e2max;
  double* scr = g.scratch + (size_t)blockIdx.x * dmax * 4 * nt + tid;
  const size_t ld = 4;                     // chain row k -> row 4k + c of its column of U

  for (;;) {
    if (tid == 0) s_atom = atomicAdd(g.counter, 1);
    __syncthreads();
    const int atom = g.atom0 + s_atom;
    if (atom >= g.n_atoms) break;
    const int K = g.kused[atom];
    const int d = 4 * K;
    const int Kp = (K + 3) & ~3;
    const double* tab = g.tab + (size_t)atom * g.r_max * 32;
    double glo = 1e300, ghi = -1e300, e2m = 0.0;
    for (int q = tid; q < 4 * Kp; q += nt) {
      const int c = q / Kp, k = q % Kp;
      double Dk = 1e30, Ek = 0.0, Em = 0.0;
      if (k < K) {
        Dk = tab[(size_t)k * 32 + 5 * c];
        Ek = (k + 1 < K) ? tab[(size_t)k * 32 + 16 + 5 * c] : 0.0;
        Em = (k > 0) ? tab[(size_t)(k - 1) * 32 + 16 + 5 * c] : 0.0;
        const double rad = fabs(Ek) + fabs(Em);
        glo = fmin(glo, Dk - rad); ghi = fmax(ghi, Dk + rad); e2m = fmax(e2m, Ek * Ek);
      }
      Dg[q] = Dk; Eg[q] = Ek; E2[q] = Ek * Ek; E2s[q] = Em * Em;
    }
    for (int off = 32; off > 0; off >>= 1) {
      glo = fmin(glo, __shfl_xor(glo, off, 64));
      ghi = fmax(ghi, __shfl_xor(ghi, off, 64));
      e2m = fmax(e2m, __shfl_xor(e2m, off, 64));
    }
    if (lane == 0) { red[wave * 4] = glo; red[wave * 4 + 1] = ghi; red[wave * 4 + 2] = e2m; }
    __syncthreads();
    if (tid == 0) {
      double a = 1e300, b = -1e300, e = 0.0;
      for (int w = 0; w < nw; ++w) { a = fmin(a, red[w * 4]); b = fmax(b, red[w * 4 + 1]); e = fmax(e, red[w * 4 + 2]); }
      const double pad = 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)) + 1e-300;
      s_lo = a - pad; s_hi = b + pad; s_e2max = e;
    }
    __syncthreads();
    const double lo0 = s_lo, hi0 = s_hi;
    const double anorm = fmax(fabs(lo0), fabs(hi0));
    const double pivmin = DBL_MIN * fmax(1.0, s_e2max);
    for (int t = tid; t < d; t += nt) {
      const int c = t / K, j = t - c * K;
      const double* Dc = Dg + c * Kp;
      const double* E2c = E2s + c * Kp;
      // the padded rows (D = 1e30) are roots far above the chain's spectrum
      lam_s[t] = eig_laguerre(Dc, E2c, Kp, j, lo0, hi0, 0, K, anorm, pivmin);
    }
    __syncthreads();
    const double ctol = fmax(1e-6 * anorm, 1e-5);
    const double small = DBL_EPSILON * anorm + 1e-300;
    int mp = 0;
    for (int t = tid; t < d; t += nt) {
      const int c0 = (t / K) * K;
      int p = 0;
      while (t - p - 1 >= c0 && lam_s[t - p] - lam_s[t - p - 1] < ctol) ++p;
      pos_s[t] = p;
      mp = p > mp ? p : mp;
    }
    for (int off = 32; off > 0; off >>= 1) { const int o = __shfl_xor(mp, off, 64); mp = o > mp ? o : mp; }
    if (tid == 0) s_maxpos = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&s_maxpos, mp);
    __syncthreads();
    const int maxpos = s_maxpos;
    UT* Ua = (UT*)g.evec + (size_t)atom * dmax * dmax;      // column t of U at Ua + t dmax
    double* vsc = g.vsc + (size_t)atom * dmax;              // normalising factor of column t
    for (int q = tid; q < d * d; q += nt) {                  // rows of the other chains
      const int t = q / d, row = q - t * d;
      if ((row & 3) != t / K) Ua[(size_t)t * dmax + row] = (UT)0.0;
    }
    for (int round = 0; round <= maxpos; ++round) {
      for (int t = tid; t < d; t += nt) {
        if (pos_s[t] != round) continue;
        const int c = t / K, cend = (c + 1) * K;
        const double* Dc = Dg + c * Kp;
        const double* Ec = Eg + c * Kp;
        const double* E2c = E2 + c * Kp;
        UT* xc = Ua + (size_t)t * dmax + c;
        if (round == 0 && (t + 1 >= cend || pos_s[t + 1] == 0)) {
          vsc[t] = twisted_ck<false, UT>(Dc, Ec, E2c, K, lam_s[t], small, xc, ld, scr, nt);
          continue;
        }
        vsc[t] = 1.0;                                // normalised here
        cluster_vector<UT>(Dc, Ec, K, lam_s[t], small, t, round, xc, ld, dmax, scr, nt);
      }
      __syncthreads();
    }
    double* lam = g.lam + (size_t)atom * dmax;
    double* wgt = g.wgt + (size_t)atom * dmax;
    double* y1 = g.y1 + (size_t)atom * 4 * dmax;
    for (int t = tid; t < dmax; t += nt) {
      const int c = t < d ? t / K : -1;
      const double a = t < d ? (double)Ua[(size_t)t * dmax + c] * vsc[t] : 0.0;   // chain row 0 = block row c
      lam[t] = t < d ? lam_s[t] : 0.0;
      wgt[t] = a * a;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) y1[(size_t)cc * dmax + t] = (cc == c) ? a : 0.0;
    }
    if (tid == 0) {
      g.ref_n[atom] = 0;
      g.seg_n[2 * atom] = 0;
      g.seg_n[2 * atom + 1] = 0;
      atomicMax((unsigned long long*)&g.stats[ST_MAX_CLUSTER_POS], (unsigned long long)maxpos);
    }
    __syncthreads();
  }
}

// Four waves per atom (the replay of the band rotations on one of them).
// VJ: element type of the rho row vectors V_J (float after the FP32 recursion).
template <typename VJ>
__global__ void __launch_bounds__(RHO_NT) k_rho(RhoArgs g) {
  extern __shared__ double rsm[];
  constexpr int NW = RHO_NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int atom = g.atom0 + blockIdx.x;
  const int dmax = 4 * g.r_max;
  double* v = rsm;                       // [dmax][4]: f(Lambda) Y[0:4,:]^T
  double* x = rsm + (size_t)dmax * 4;    // row m at xrow(m)
  const double mu = g.mu_state[2];
  const int d = 4 * g.kused[atom];
  {
    const double* lam = g.lam + (size_t)atom * dmax;
    const double* y1 = g.y1 + (size_t)atom * 4 * dmax;
    const double* vsc = g.vsc + (size_t)atom * dmax;     // U is stored with unnormalised columns
    for (int q = tid; q < 4 * d; q += RHO_NT) {
      const int m = q >> 2, col = q & 3;
      const double z = (lam[m] - mu) / g.kT;
      const double e = exp(-fabs(z));
      const double f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
      v[q] = f * y1[(size_t)col * dmax + m] * vsc[m];
    }
  }
  __syncthreads();
  // x = U v (eigenvectors of the tridiagonal): one row of x per thread, over
  // the columns of U (stored column by column: the lanes read consecutive
  // rows of a column), v_m broadcast from LDS
  const VJ* Ua = (const VJ*)g.evec + (size_t)atom * dmax * dmax;   // U in the recursion's precision
  for (int k = tid; k < d; k += RHO_NT) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
    for (int m = 0; m < d; ++m) {
      const double u = (double)Ua[(size_t)m * dmax + k];
      a0 += u * v[4 * m]; a1 += u * v[4 * m + 1]; a2 += u * v[4 * m + 2]; a3 += u * v[4 * m + 3];
    }
    double* xk = x + xrow(k);
    xk[0] = a0; xk[1] = a1; xk[2] = a2; xk[3] = a3;
  }
  __syncthreads();
  // c = Z x: the reflector segments in reverse; the reflectors of one segment
  // commute. One wave replays them: the segment table is staged in LDS, the
  // reflector log in windows (coalesced loads), and the segments are ordered
  // by wave-scope fences. Rows d .. d+3 of x are zero (windows at the end
  // reach them; their reflector entries are zero).
  if (wave == 0) {
    const double* lv = g.ref_v + (size_t)atom * g.ref_max * 4;
    const uint16_t* lp = g.ref_p + (size_t)atom * g.ref_max;
    const int* seg = g.seg + (size_t)atom * g.seg_max;
    const int nref = g.ref_n[atom];
    const int nb = g.seg_n[2 * atom];
    int* s_seg = (int*)(x + xrow(dmax + 3) + 4);                        // [seg_max]
    double* s_v = (double*)(s_seg + ((g.seg_max + 3) & ~3));            // [RHO_REFW][4]
    uint16_t* s_p = (uint16_t*)(s_v + 4 * RHO_REFW);                    // [RHO_REFW]
    for (int q = lane; q < 16; q += 64) x[xrow(d + (q >> 2)) + (q & 3)] = 0.0;
    for (int q = lane; q < nb; q += 64) s_seg[q] = seg[q];
    auto wave_sync = [] {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    wave_sync();
    int k = nb - 1;
    while (k >= 0) {
      const int en = (k + 1 < nb) ? s_seg[k + 1] : nref;
      // the window: segments kw .. k whose reflectors fit in RHO_REFW (at least one)
      int kw = k;
      for (int base = k; base >= 0; base -= 64) {
        const int qq = base - lane;
        const bool fits = qq >= 0 && en - s_seg[qq] <= RHO_REFW;
        const uint64_t msk = __ballot(fits);
        // lanes are ordered by decreasing qq; the fitting ones form a prefix
        const int nfit = __popcll(msk);
        if (nfit > 0) kw = base - nfit + 1;
        if (nfit < 64) break;
      }
      const int w0 = s_seg[kw];
      if (en - w0 > RHO_REFW) {       // one segment with more reflectors than the window: not
        if (lane == 0)                // reached for d <= 1024 (at most 2 (d / 11 + 1) per segment)
          atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_REFLOG_OVERFLOW);
        break;
      }
      for (int e = w0 + lane; e < en; e += 64) {
        *(double4*)(s_v + 4 * (size_t)(e - w0)) = *(const double4*)(lv + 4 * (size_t)e);
        s_p[e - w0] = lp[e];
      }
      wave_sync();
      for (int kk = k; kk >= kw; --kk) {
        const int st = s_seg[kk] - w0;
        const int se = (kk == k ? en : s_seg[kk + 1]) - w0;
        for (int e = st + lane; e < se; e += 64) {
          const double4 vt = *(const double4*)(s_v + 4 * (size_t)e);
          const int p0 = s_p[e];
          double* x0 = x + xrow(p0);
          double* x1 = x + xrow(p0 + 1);
          double* x2 = x + xrow(p0 + 2);
          double* x3 = x + xrow(p0 + 3);
          double a0[4], a1[4], a2[4], a3[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) { a0[c] = x0[c]; a1[c] = x1[c]; a2[c] = x2[c]; a3[c] = x3[c]; }
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double f = vt.w * (a0[c] + vt.x * a1[c] + vt.y * a2[c] + vt.z * a3[c]);
            x0[c] = a0[c] - f;
            x1[c] = a1[c] - f * vt.x;
            x2[c] = a2[c] - f * vt.y;
            x3[c] = a3[c] - f * vt.z;
          }
        }
        wave_sync();
      }
      k = kw - 1;
    }
  }
  __syncthreads();
  // rho_{J,i}[4 js + a][col] = sum_m V_J[4 js + a][m] x[m][col]: four rows of
  // V_J at a time per wave, read along the row by the lanes, reduced over the
  // wave
  const int nJ = 1 + g.hop_n[atom];
  const int64_t p0 = g.row_ptr[atom];
  const int vld = 4 * g.r_max;
  for (int q0 = 4 * wave; q0 < 4 * nJ; q0 += 4 * NW) {
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const size_t row0 = (size_t)atom * (4 * (g.zmax + 1)) + q0;
    for (int m = lane; m < d; m += 64) {
      const double* xm = x + xrow(m);
      const double x0 = xm[0], x1 = xm[1], x2 = xm[2], x3 = xm[3];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double vv = (double)((const VJ*)g.vj)[(row0 + r) * vld + m];
        acc[r * 4] += vv * x0; acc[r * 4 + 1] += vv * x1; acc[r * 4 + 2] += vv * x2; acc[r * 4 + 3] += vv * x3;
      }
    }
    int which;
    const double sum = wave_sum16(acc, lane, which);
    // rows q0 .. q0+3 are the four orbital rows of row atom q0 / 4
    if ((lane & 3) == 0) g.rho[(size_t)(p0 + (q0 >> 2)) * 16 + which] = sum;
  }
}

size_t eig_lds_bytes(int r_max) {
  const size_t dmax = 4 * (size_t)r_max;
  const size_t band = (4 * dmax + 5 * dmax) * sizeof(double) + 4 * (EIG_NT / 64) * sizeof(double) +
                      (dmax + EIG_NT) * sizeof(int) + 64;
  const size_t dp = 4 * (size_t)((r_max + 3) & ~3);          // k_eig_chains
  const size_t chains = (4 * dp + dmax + 4 * (EIG_NT / 64)) * sizeof(double) + dmax * sizeof(int) + 64;
  return band > chains ? band : chains;
}
size_t band_lds_bytes(int r_max) {
  const size_t nc = (size_t)band_cols(4 * r_max);
  return (nc * SBR_LS + 4 * (nc | 1)) * sizeof(double) + 64;
}
size_t rho_lds_bytes(int r_max) {
  const int dmax = 4 * r_max;
  const size_t segs = ((size_t)band_segments(dmax) + 3) & ~(size_t)3;
  return ((size_t)dmax * 4 + xrow(dmax + 3) + 4) * sizeof(double) + segs * sizeof(int) +
         RHO_REFW * (4 * sizeof(double) + 2) + 64;
}
// Threads of a k_eig workgroup: one per eigenvalue of the largest T.
int eig_threads(int r_max) {
  const int t = 64 * ((4 * r_max + 63) / 64);
  return t < EIG_NT ? t : EIG_NT;
}

hipError_t eig_set_lds(int r_max) {
  const void* eig_fn[4] = {(const void*)k_eig<double>, (const void*)k_eig<float>,
                           (const void*)k_eig_chains<double>, (const void*)k_eig_chains<float>};
  hipError_t e = hipSuccess;
  for (int q = 0; q < 4; ++q) {
    e = hipFuncSetAttribute(eig_fn[q], hipFuncAttributeMaxDynamicSharedMemorySize, (int)eig_lds_bytes(r_max));
    if (e != hipSuccess) return e;
  }
  e = hipFuncSetAttribute((const void*)k_band, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)band_lds_bytes(r_max));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_rho<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)rho_lds_bytes(r_max));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_rho<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)rho_lds_bytes(r_max));
}

void launch_eig(const EigArgs& a, int n_wg, hipStream_t st) {
  if (a.scalar) {
    if (a.u_fp32)
      hipLaunchKernelGGL(k_eig_chains<float>, dim3(n_wg), dim3(eig_threads(a.r_max)), eig_lds_bytes(a.r_max), st, a);
    else
      hipLaunchKernelGGL(k_eig_chains<double>, dim3(n_wg), dim3(eig_threads(a.r_max)), eig_lds_bytes(a.r_max), st, a);
    return;
  }
  hipLaunchKernelGGL(k_band, dim3(a.n_atoms - a.atom0), dim3(BAND_NT), band_lds_bytes(a.r_max), st, a);
  if (a.u_fp32) hipLaunchKernelGGL(k_eig<float>, dim3(n_wg), dim3(eig_threads(a.r_max)), eig_lds_bytes(a.r_max), st, a);
  else hipLaunchKernelGGL(k_eig<double>, dim3(n_wg), dim3(eig_threads(a.r_max)), eig_lds_bytes(a.r_max), st, a);
}
void launch_rho(const RhoArgs& a, hipStream_t st) {
  if (a.vj_fp32) hipLaunchKernelGGL(k_rho<float>, dim3(a.n_atoms - a.atom0), dim3(RHO_NT), rho_lds_bytes(a.r_max), st, a);
  else hipLaunchKernelGGL(k_rho<double>, dim3(a.n_atoms - a.atom0), dim3(RHO_NT), rho_lds_bytes(a.r_max), st, a);
}

}  // namespace tbk
