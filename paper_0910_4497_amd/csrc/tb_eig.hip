// Projected eigenproblem and density-matrix assembly (Sec. 3: the small
// projected matrix is diagonalised; Sec. 2, Eq. 2: rho = sum |m> f <m|).
//
// k_eig (one wave per atom, FP64): T (block tridiagonal, 4x4 blocks A_k,
// upper-triangular B_k, so a symmetric band of half-width 4) is reduced to
// tridiagonal form by Givens rotations that chase the fill-in ("bulge") down
// the band, then diagonalised by the implicit QL iteration with Wilkinson
// shifts (Bowdler, Martin, Reinsch & Wilkinson, 1968). Every plane rotation
// is applied to the first four rows of the accumulated eigenvector matrix
// (they give Y[0:4, :], hence the seed weights w_m) and logged (c, s, plane).
//
// k_rho (one wave per atom): after the chemical potential is known,
// c = Y f(Lambda) Y[0:4, :]^T is obtained by replaying the logged rotations
// in reverse on the 4r x 4 block f(Lambda) Y[0:4, :]^T (no eigenvector matrix
// is ever stored), and rho_{J,i} = V_J c for the rho row atoms J.
//
// Rotation convention: a logged (c, s, p) acts on the column pair (p, p+1)
// of a row vector set R as R_p <- c R_p + s R_{p+1}, R_{p+1} <- -s R_p + c R_{p+1}
// (R <- R G^T); Y is the ordered product of all these, so Y x is the reverse
// replay x_p <- c x_p - s x_{p+1}, x_{p+1} <- s x_p + c x_{p+1}.
#include <float.h>

#include "tb_internal.h"

namespace tbk {

constexpr int EIG_NT = 64;
constexpr int BW = 4;              // half-bandwidth of T
constexpr int LB = BW + 2;         // stored lower diagonals incl. the bulge


__device__ __forceinline__ double t_entry(const double* tab, int row, int col) {
  // lower triangle (row >= col) of the block tridiagonal T
  const int kr = row >> 2, ar = row & 3, kc = col >> 2, ac = col & 3;
  if (kr == kc) return tab[(size_t)kc * 32 + ar * 4 + ac];
  if (kr == kc + 1) return (ar <= ac) ? tab[(size_t)kc * 32 + 16 + ar * 4 + ac] : 0.0;
  return 0.0;
}

// Givens pair from (x, y): r = hypot(x, y), c = x / r, s = y / r.
__device__ __forceinline__ void givens(double x, double y, double& c, double& s, double& r) {
  const double q = x * x + y * y;
  if (q == 0.0) { c = 1.0; s = 0.0; r = 0.0; return; }
  const double inv = rsqrt(q);
  c = x * inv; s = y * inv; r = q * inv;
}

// Band -> tridiagonal, one diagonal at a time (half-width bc -> bc - 1 for
// bc = 4, 3, 2). For every column j the element at offset bc is zeroed by a
// rotation in plane (j+bc-1, j+bc); the fill-in it creates at offset bc+1 is
// chased down the band in steps of bc. Chase j starts at time j * I and moves
// one rotation per time step; with I * bc - 1 >= bc + 3 the rotations of
// concurrent chases touch disjoint entries, so every time step applies one
// rotation per active chase (one thread each) and the result equals the
// sequential column-by-column order.
__global__ void __launch_bounds__(EIG_NT) k_eig(EigArgs g) {
  extern __shared__ double esm[];
  const int atom = blockIdx.x, lane = threadIdx.x;
  const int dmax = 4 * g.r_max;
  double* Lb = esm;                      // [dmax][LB]: Lb[j][t] = T[j+t][j]
  double* R1 = esm + (size_t)dmax * LB;  // [4][d]
  const int K = g.kused[atom];
  const int d = 4 * K;
  const double* tab = g.tab + (size_t)atom * g.r_max * 32;
  for (int q = lane; q < d * LB; q += EIG_NT) {
    const int j = q / LB, t = q % LB;
    const int row = j + t;
    Lb[q] = (t <= BW && row < d) ? t_entry(tab, row, j) : 0.0;
  }
  for (int q = lane; q < 4 * d; q += EIG_NT) {
    const int c = q / d, m = q % d;
    R1[q] = (m == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  double* lcs = g.rot_cs + (size_t)atom * g.rot_max * 2;
  uint16_t* lp = g.rot_p + (size_t)atom * g.rot_max;
  int64_t nrot = 0;
  bool overflow = false;
  int* seg = g.seg + (size_t)atom * g.seg_max;
  int nseg = 0;

  // ---- band -> tridiagonal, pipelined chases (one thread per chase)
  for (int bc = BW; bc >= 2; --bc) {
    const int I = (bc + 4 + bc - 1) / bc;           // ceil((bc + 4) / bc): 2, 3, 3
    const int nchase = d - bc;
    if (nchase <= 0) continue;
    const int last = nchase - 1;
    const int t_end = last * I + (d - 1 - last - bc) / bc + 1;
    for (int tau = 0; tau < t_end; ++tau) {
      int jtop = tau / I;
      if (jtop > last) jtop = last;
      const int64_t step_start = nrot;
      // chases jtop, jtop-1, ... in batches of 64 until one has finished
      // (every smaller j started earlier and is finished too)
      for (int jb = jtop; jb >= 0; jb -= EIG_NT) {
        const int j = jb - lane;
        bool act = false;
        int p = 0, m0 = 0;
        if (j >= 0) {
          const int st = tau - j * I;
          p = j + bc - 1 + st * bc;
          act = (p + 1 <= d - 1);
          m0 = (st == 0) ? p + 1 - bc : p - bc;
        }
        const bool batch_done = __ballot(act) == 0ull;
        double x = 0.0, y = 0.0;
        if (act) {
          x = Lb[(size_t)m0 * LB + (p - m0)];
          y = Lb[(size_t)m0 * LB + (p + 1 - m0)];
          act = (y != 0.0);
        }
        double c = 1.0, s = 0.0, r = 0.0;
        if (act) {
          givens(x, y, c, s, r);
          const int q = p + 1;
          // left pairs (T[p][m], T[q][m]), m in [p - bc, p - 1]
          for (int m = (p - bc > 0 ? p - bc : 0); m < p; ++m) {
            double* up = Lb + (size_t)m * LB + (p - m);
            double* uq = Lb + (size_t)m * LB + (q - m);
            const double u = *up, v = *uq;
            if (m == m0) { *up = r; *uq = 0.0; }
            else { *up = c * u + s * v; *uq = -s * u + c * v; }
          }
          // right pairs (T[m][p], T[m][q]), m in [p + 2, p + 1 + bc]
          const int mr = (p + 1 + bc < d - 1) ? p + 1 + bc : d - 1;
          for (int m = p + 2; m <= mr; ++m) {
            double* up = Lb + (size_t)p * LB + (m - p);
            double* uq = Lb + (size_t)q * LB + (m - q);
            const double u = *up, v = *uq;
            *up = c * u + s * v; *uq = -s * u + c * v;
          }
          // 2x2 diagonal block
          {
            const double a = Lb[(size_t)p * LB], b = Lb[(size_t)p * LB + 1], e = Lb[(size_t)q * LB];
            const double cc = c * c, ss = s * s, cs = c * s;
            Lb[(size_t)p * LB] = cc * a + 2.0 * cs * b + ss * e;
            Lb[(size_t)q * LB] = ss * a - 2.0 * cs * b + cc * e;
            Lb[(size_t)p * LB + 1] = cs * (e - a) + (cc - ss) * b;
          }
          // first four rows of the accumulated transform
#pragma unroll
          for (int row = 0; row < 4; ++row) {
            double* rr = R1 + (size_t)row * d;
            const double u = rr[p], v = rr[q];
            rr[p] = c * u + s * v; rr[q] = -s * u + c * v;
          }
        }
        // log in lane order (rotations of one time step commute)
        const uint64_t mask = __ballot(act);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int64_t slot = nrot + __popcll(mask & below);
        if (act && slot < g.rot_max) { lcs[2 * slot] = c; lcs[2 * slot + 1] = s; lp[slot] = (uint16_t)p; }
        nrot += __popcll(mask);
        if (batch_done) break;
      }
      if (nrot > step_start) {                    // one segment per non-empty time step
        if (lane == 0 && nseg < g.seg_max) seg[nseg] = (int)step_start;
        ++nseg;
      }
      __syncthreads();
    }
  }
  const int nseg_band = nseg;
  if (nrot > g.rot_max) { overflow = true; nrot = g.rot_max; }

  // ---- implicit QL on the tridiagonal: D[j] = Lb[j][0], E[j] = Lb[j][1]
  // Every lane runs the scalar recursion; lanes 0..3 carry one row of R1,
  // lane 4 writes the log. Within a sweep no entry is read after being
  // written, so the sweep needs no barrier; the next entries are prefetched.
  int max_it = 0;
  bool noconv = false;
  for (int l = 0; l < d; ++l) {
    int it = 0;
    for (;;) {
      // first m >= l with a negligible E[m] (m = d-1 if none), 64 at a time
      int m = d - 1;
      for (int base = l; base < d - 1; base += EIG_NT) {
        const int mm = base + lane;
        bool neg = true;
        if (mm < d - 1) {
          const double dd = fabs(Lb[(size_t)mm * LB]) + fabs(Lb[(size_t)(mm + 1) * LB]);
          neg = (fabs(Lb[(size_t)mm * LB + 1]) + dd == dd);
        }
        const uint64_t bm = __ballot(neg);
        if (bm) { m = base + __ffsll((unsigned long long)bm) - 1; break; }
      }
      if (m == l) break;
      if (it == 60) { noconv = true; break; }
      ++it;
      if (lane == 0 && nseg < g.seg_max) seg[nseg] = (int)nrot;   // one segment per sweep
      ++nseg;
      const double Dl = Lb[(size_t)l * LB], El = Lb[(size_t)l * LB + 1];
      double gg = (Lb[(size_t)(l + 1) * LB] - Dl) / (2.0 * El);
      double rr = sqrt(gg * gg + 1.0);
      gg = Lb[(size_t)m * LB] - Dl + El / (gg + copysign(rr, gg));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool underflow = false;
      const int row = lane < 4 ? lane : 0;
      double carry = R1[(size_t)row * d + m];
      double Ei = Lb[(size_t)i * LB + 1], Di = Lb[(size_t)i * LB], Di1 = Lb[(size_t)m * LB];
      double Ri = R1[(size_t)row * d + i];
      for (; i >= l; --i) {
        // prefetch the next iteration's inputs (entries not written in this sweep)
        const int in = i > l ? i - 1 : i;
        const double En = Lb[(size_t)in * LB + 1], Dn = Lb[(size_t)in * LB];
        const double Rn = R1[(size_t)row * d + in];
        const double f = s * Ei, b = c * Ei;
        const double q2 = f * f + gg * gg;
        if (q2 == 0.0) {
          if (lane == 0) { Lb[(size_t)(i + 1) * LB + 1] = 0.0; Lb[(size_t)(i + 1) * LB] = Di1 - p; Lb[(size_t)m * LB + 1] = 0.0; }
          underflow = true;
          break;
        }
        const double inv = rsqrt(q2);
        rr = q2 * inv;
        s = f * inv; c = gg * inv;
        gg = Di1 - p;
        rr = (Di - gg) * s + 2.0 * c * b;
        p = s * rr;
        const double Dnew = gg + p;
        gg = c * rr - b;
        if (lane == 0) { Lb[(size_t)(i + 1) * LB + 1] = q2 * inv; Lb[(size_t)(i + 1) * LB] = Dnew; }
        if (lane < 4) R1[(size_t)row * d + (i + 1)] = s * Ri + c * carry;
        carry = c * Ri - s * carry;
        if (lane == 4 && nrot < g.rot_max) { lcs[2 * nrot] = c; lcs[2 * nrot + 1] = -s; lp[nrot] = (uint16_t)i; }
        if (nrot < g.rot_max) ++nrot; else overflow = true;
        Ei = En; Di1 = Di; Di = Dn; Ri = Rn;
      }
      if (lane < 4) R1[(size_t)row * d + (i + 1)] = carry;
      __syncthreads();
      if (underflow && i >= l) continue;
      if (lane == 0) {
        Lb[(size_t)l * LB] -= p;
        Lb[(size_t)l * LB + 1] = gg;
        Lb[(size_t)m * LB + 1] = 0.0;
      }
      __syncthreads();
    }
    if (it > max_it) max_it = it;
  }
  __syncthreads();
  // ---- outputs (padding beyond d: lambda = 0, w = 0, Y1 = 0)
  double* lam = g.lam + (size_t)atom * dmax;
  double* wgt = g.wgt + (size_t)atom * dmax;
  double* y1 = g.y1 + (size_t)atom * 4 * dmax;
  for (int m = lane; m < dmax; m += EIG_NT) {
    if (m < d) {
      const double a0 = R1[m], a1 = R1[(size_t)d + m], a2 = R1[(size_t)2 * d + m], a3 = R1[(size_t)3 * d + m];
      lam[m] = Lb[(size_t)m * LB];
      wgt[m] = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
      y1[m] = a0; y1[dmax + m] = a1; y1[2 * dmax + m] = a2; y1[3 * dmax + m] = a3;
    } else {
      lam[m] = 0.0; wgt[m] = 0.0;
      y1[m] = 0.0; y1[dmax + m] = 0.0; y1[2 * dmax + m] = 0.0; y1[3 * dmax + m] = 0.0;
    }
  }
  if (lane == 0) {
    g.rot_n[atom] = (int)(nrot < g.rot_max ? nrot : g.rot_max);
    g.seg_n[2 * atom] = nseg_band;
    g.seg_n[2 * atom + 1] = nseg < g.seg_max ? nseg : g.seg_max;
    if (nseg > g.seg_max) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_SEG_OVERFLOW);
    atomicMax((unsigned long long*)&g.stats[ST_MAX_EIG_ITERS], (unsigned long long)max_it);
    if (noconv) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_EIG_NOCONV);
    if (overflow) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_ROTLOG_OVERFLOW);
  }
}

// Reverse replay, one wave per atom, x = f(Lambda) Y[0:4,:]^T (4r x 4) in LDS.
//  1. QL sweeps, last first. Sweep s logged planes m_s-1, ..., l_s (one chain);
//     its replay runs l_s upward. Replayed sweep r starts at time 2r, so it
//     trails the previous one by two planes: l never decreases from one forward
//     sweep to the next, which keeps concurrent rotations on disjoint rows and
//     every row's updates in the sequential reverse order.
//  2. band steps, last first; rotations of one step commute (disjoint rows).
__global__ void __launch_bounds__(EIG_NT) k_rho(RhoArgs g) {
  extern __shared__ double rsm[];
  const int lane = threadIdx.x;
  const int atom = blockIdx.x;
  const int dmax = 4 * g.r_max;
  double* x = rsm;                       // [dmax][4]
  const double mu = g.mu_state[2];
  const int d = 4 * g.kused[atom];
  {
    const double* lam = g.lam + (size_t)atom * dmax;
    const double* y1 = g.y1 + (size_t)atom * 4 * dmax;
    for (int q = lane; q < 4 * d; q += EIG_NT) {
      const int m = q >> 2, col = q & 3;
      const double z = (lam[m] - mu) / g.kT;
      const double e = exp(-fabs(z));
      const double f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
      x[q] = f * y1[(size_t)col * dmax + m];
    }
  }
  const double* lcs = g.rot_cs + (size_t)atom * g.rot_max * 2;
  const uint16_t* lp = g.rot_p + (size_t)atom * g.rot_max;
  const int* seg = g.seg + (size_t)atom * g.seg_max;
  const int nrot = g.rot_n[atom];
  const int nb = g.seg_n[2 * atom], ns = g.seg_n[2 * atom + 1];
  const int S = ns - nb;                           // QL sweeps
  auto seg_end = [&](int k) { return k + 1 < ns ? seg[k + 1] : nrot; };
  __syncthreads();
  // ---- 1. QL sweeps, pipelined
  int maxlen = 0;
  for (int k = nb + lane; k < ns; k += EIG_NT) { const int len = seg_end(k) - seg[k]; maxlen = len > maxlen ? len : maxlen; }
  for (int off = 32; off > 0; off >>= 1) { const int o = __shfl_xor(maxlen, off, 64); maxlen = o > maxlen ? o : maxlen; }
  const int t_end = S > 0 ? 2 * (S - 1) + maxlen : 0;
  for (int tau = 0; tau < t_end; ++tau) {
    // replayed sweep r (forward sweep s = nb + S - 1 - r) is at rotation tau - 2r
    int rhi = tau / 2;
    if (rhi > S - 1) rhi = S - 1;
    int rlo = (tau - maxlen + 2) / 2;
    if (rlo < 0) rlo = 0;
    for (int r = rhi - lane; r >= rlo; r -= EIG_NT) {
      const int k = nb + S - 1 - r;
      const int st = seg[k], en = seg_end(k);
      const int t = tau - 2 * r;
      if (t < en - st) {
        const int e = en - 1 - t;
        const double c = lcs[2 * e], s = lcs[2 * e + 1];
        const int p = lp[e];
        double* xp = x + 4 * p;
        const double a0 = xp[0], a1 = xp[1], a2 = xp[2], a3 = xp[3];
        const double b0 = xp[4], b1 = xp[5], b2 = xp[6], b3 = xp[7];
        xp[0] = c * a0 - s * b0; xp[1] = c * a1 - s * b1; xp[2] = c * a2 - s * b2; xp[3] = c * a3 - s * b3;
        xp[4] = s * a0 + c * b0; xp[5] = s * a1 + c * b1; xp[6] = s * a2 + c * b2; xp[7] = s * a3 + c * b3;
      }
    }
    __syncthreads();
  }
  // ---- 2. band steps, last first
  for (int k = nb - 1; k >= 0; --k) {
    const int st = seg[k], en = seg_end(k);
    for (int e = st + lane; e < en; e += EIG_NT) {
      const double c = lcs[2 * e], s = lcs[2 * e + 1];
      const int p = lp[e];
      double* xp = x + 4 * p;
      const double a0 = xp[0], a1 = xp[1], a2 = xp[2], a3 = xp[3];
      const double b0 = xp[4], b1 = xp[5], b2 = xp[6], b3 = xp[7];
      xp[0] = c * a0 - s * b0; xp[1] = c * a1 - s * b1; xp[2] = c * a2 - s * b2; xp[3] = c * a3 - s * b3;
      xp[4] = s * a0 + c * b0; xp[5] = s * a1 + c * b1; xp[6] = s * a2 + c * b2; xp[7] = s * a3 + c * b3;
    }
    __syncthreads();
  }
  // ---- rho_{J,i}[4 js + a][col] = sum_m V_J[4 js + a][m] x[m][col]
  const int nJ = 1 + g.hop_n[atom];
  const int64_t p0 = g.row_ptr[atom];
  const int vld = 4 * g.r_max;
  for (int q = lane; q < 4 * nJ; q += EIG_NT) {
    const size_t row = (size_t)atom * (4 * JMAX) + q;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (g.vj_fp32) {
      const float* vr = (const float*)g.vj + row * vld;
      for (int m = 0; m < d; ++m) {
        const double v = vr[m];
        s0 += v * x[4 * m]; s1 += v * x[4 * m + 1]; s2 += v * x[4 * m + 2]; s3 += v * x[4 * m + 3];
      }
    } else {
      const double* vr = (const double*)g.vj + row * vld;
      for (int m = 0; m < d; ++m) {
        const double v = vr[m];
        s0 += v * x[4 * m]; s1 += v * x[4 * m + 1]; s2 += v * x[4 * m + 2]; s3 += v * x[4 * m + 3];
      }
    }
    double* out = g.rho + (size_t)(p0 + (q >> 2)) * 16 + (q & 3) * 4;
    out[0] = s0; out[1] = s1; out[2] = s2; out[3] = s3;
  }
}

size_t eig_lds_bytes(int r_max) { return (size_t)4 * r_max * (LB + 4) * sizeof(double); }
size_t rho_lds_bytes(int r_max) { return (size_t)4 * r_max * 4 * sizeof(double); }

hipError_t eig_set_lds(int r_max) {
  hipError_t e = hipFuncSetAttribute((const void*)k_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)eig_lds_bytes(r_max));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_rho, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)rho_lds_bytes(r_max));
}

void launch_eig(const EigArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_eig, dim3(a.n_atoms), dim3(EIG_NT), eig_lds_bytes(a.r_max), st, a);
}
void launch_rho(const RhoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_rho, dim3(a.n_atoms), dim3(EIG_NT), rho_lds_bytes(a.r_max), st, a);
}

}  // namespace tbk
