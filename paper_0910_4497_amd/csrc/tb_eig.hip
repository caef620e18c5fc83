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

__global__ void __launch_bounds__(EIG_NT) k_eig(EigArgs g) {
  extern __shared__ double esm[];
  const int atom = blockIdx.x, lane = threadIdx.x;
  const int dmax = 4 * g.r_max;
  double* Lb = esm;                      // [dmax][LB]: Lb[j][t] = T[j+t][j]
  double* R1 = esm + (size_t)dmax * LB;  // [4][dmax]
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

  // Rotation in plane (p, p+1) that zeroes T[p+1][col] against T[p][col].
  auto band_rotate = [&](int p, int col) {
    const int q = p + 1;
    const double x = Lb[(size_t)col * LB + (p - col)];
    const double y = Lb[(size_t)col * LB + (q - col)];
    const double r = sqrt(x * x + y * y);
    const double c = x / r, s = y / r;
    if (lane < 4) {                       // left columns m in [p-4, p-1]
      const int m = p - 4 + lane;
      if (m >= 0) {
        double* up = Lb + (size_t)m * LB + (p - m);
        double* uq = Lb + (size_t)m * LB + (q - m);
        const double u = *up, v = *uq;
        if (m == col) { *up = r; *uq = 0.0; }
        else { *up = c * u + s * v; *uq = -s * u + c * v; }
      }
    } else if (lane < 8) {                // right rows m in [q+1, q+4]
      const int m = q + 1 + (lane - 4);
      if (m < d) {
        double* up = Lb + (size_t)p * LB + (m - p);
        double* uq = Lb + (size_t)q * LB + (m - q);
        const double u = *up, v = *uq;
        *up = c * u + s * v; *uq = -s * u + c * v;
      }
    } else if (lane == 8) {               // 2x2 diagonal block
      const double a = Lb[(size_t)p * LB], b = Lb[(size_t)p * LB + 1], e = Lb[(size_t)q * LB];
      const double cc = c * c, ss = s * s, cs = c * s;
      Lb[(size_t)p * LB] = cc * a + 2.0 * cs * b + ss * e;
      Lb[(size_t)q * LB] = ss * a - 2.0 * cs * b + cc * e;
      Lb[(size_t)p * LB + 1] = cs * (e - a) + (cc - ss) * b;
    } else if (lane < 13) {               // first four rows of the eigenvector matrix
      double* rr = R1 + (size_t)(lane - 9) * d;
      const double u = rr[p], v = rr[q];
      rr[p] = c * u + s * v; rr[q] = -s * u + c * v;
    } else if (lane == 13) {
      if (nrot < g.rot_max) { lcs[2 * nrot] = c; lcs[2 * nrot + 1] = s; lp[nrot] = (uint16_t)p; }
    }
    if (nrot < g.rot_max) ++nrot; else overflow = true;
    __syncthreads();
  };

  // ---- band -> tridiagonal
  for (int j = 0; j + 2 < d; ++j) {
    for (int t = BW; t >= 2; --t) {
      const int i = j + t;
      if (i >= d) continue;
      if (Lb[(size_t)j * LB + t] == 0.0) continue;
      band_rotate(i - 1, j);
      int pp = i - 1;                      // bulge now at (pp + BW + 1, pp)
      while (pp + BW + 1 < d) {
        if (Lb[(size_t)pp * LB + BW + 1] == 0.0) break;
        band_rotate(pp + BW, pp);
        pp += BW;
      }
    }
  }
  __syncthreads();

  // ---- implicit QL on the tridiagonal: D[j] = Lb[j][0], E[j] = Lb[j][1]
  int max_it = 0;
  bool noconv = false;
  for (int l = 0; l < d; ++l) {
    int it = 0;
    for (;;) {
      int m = l;
      for (; m < d - 1; ++m) {
        const double dd = fabs(Lb[(size_t)m * LB]) + fabs(Lb[(size_t)(m + 1) * LB]);
        if (fabs(Lb[(size_t)m * LB + 1]) + dd == dd) break;
      }
      if (m == l) break;
      if (it == 60) { noconv = true; break; }
      ++it;
      const double Dl = Lb[(size_t)l * LB], El = Lb[(size_t)l * LB + 1];
      double gg = (Lb[(size_t)(l + 1) * LB] - Dl) / (2.0 * El);
      double rr = sqrt(gg * gg + 1.0);
      gg = Lb[(size_t)m * LB] - Dl + El / (gg + copysign(rr, gg));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool underflow = false;
      // carried value of column i+1 of R1 (lanes 0..3)
      double carry = (lane < 4) ? R1[(size_t)lane * d + m] : 0.0;
      for (; i >= l; --i) {
        const double Ei = Lb[(size_t)i * LB + 1], Di = Lb[(size_t)i * LB];
        const double Di1 = Lb[(size_t)(i + 1) * LB];
        const double f = s * Ei, b = c * Ei;
        rr = sqrt(f * f + gg * gg);
        if (lane == 0) Lb[(size_t)(i + 1) * LB + 1] = rr;
        if (rr == 0.0) {
          if (lane == 0) { Lb[(size_t)(i + 1) * LB] = Di1 - p; Lb[(size_t)m * LB + 1] = 0.0; }
          underflow = true;
          break;
        }
        const double inv = 1.0 / rr;
        s = f * inv; c = gg * inv;
        gg = Di1 - p;
        rr = (Di - gg) * s + 2.0 * c * b;
        p = s * rr;
        if (lane == 0) Lb[(size_t)(i + 1) * LB] = gg + p;
        gg = c * rr - b;
        if (lane < 4) {
          const double u = R1[(size_t)lane * d + i];
          R1[(size_t)lane * d + (i + 1)] = s * u + c * carry;
          carry = c * u - s * carry;
        } else if (lane == 4) {
          if (nrot < g.rot_max) { lcs[2 * nrot] = c; lcs[2 * nrot + 1] = -s; lp[nrot] = (uint16_t)i; }
        }
        if (nrot < g.rot_max) ++nrot; else overflow = true;
        __syncthreads();
      }
      if (lane < 4) R1[(size_t)lane * d + (i + 1)] = carry;
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
    atomicMax((unsigned long long*)&g.stats[ST_MAX_EIG_ITERS], (unsigned long long)max_it);
    if (noconv) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_EIG_NOCONV);
    if (overflow) atomicOr((unsigned long long*)&g.stats[ST_FLAGS], (unsigned long long)FL_ROTLOG_OVERFLOW);
  }
}


__global__ void __launch_bounds__(EIG_NT) k_rho(RhoArgs g) {
  extern __shared__ double rsm[];
  const int atom = blockIdx.x, lane = threadIdx.x;
  const int dmax = 4 * g.r_max;
  const int d = 4 * g.kused[atom];
  double* x = rsm;                      // [dmax][4]
  const double mu = g.mu_state[2];
  const double* lam = g.lam + (size_t)atom * dmax;
  const double* y1 = g.y1 + (size_t)atom * 4 * dmax;
  for (int q = lane; q < 4 * d; q += EIG_NT) {
    const int m = q >> 2, b = q & 3;
    const double z = (lam[m] - mu) / g.kT;
    const double e = exp(-fabs(z));
    const double f = (z > 0.0) ? 2.0 * e / (1.0 + e) : 2.0 / (1.0 + e);
    x[q] = f * y1[(size_t)b * dmax + m];
  }
  __syncthreads();
  const int nrot = g.rot_n[atom];
  const double* lcs = g.rot_cs + (size_t)atom * g.rot_max * 2;
  const uint16_t* lp = g.rot_p + (size_t)atom * g.rot_max;
  // reverse replay, 64 log entries staged per lane at a time
  for (int base = nrot - 1; base >= 0; base -= EIG_NT) {
    const int t = base - lane;
    double mc = 1.0, ms = 0.0;
    int mp = 0;
    if (t >= 0) { mc = lcs[2 * t]; ms = lcs[2 * t + 1]; mp = lp[t]; }
    const int cnt = base + 1 < EIG_NT ? base + 1 : EIG_NT;
    for (int u = 0; u < cnt; ++u) {
      const double c = __shfl(mc, u, 64), s = __shfl(ms, u, 64);
      const int p = __shfl(mp, u, 64);
      if (lane < 4) {
        const double a = x[4 * p + lane], b = x[4 * (p + 1) + lane];
        x[4 * p + lane] = c * a - s * b;
        x[4 * (p + 1) + lane] = s * a + c * b;
      }
      __syncthreads();
    }
  }
  // rho_{J,i} = V_J c
  const int nJ = 1 + g.hop_n[atom];
  const int64_t p0 = g.row_ptr[atom];
  const int vld = 4 * g.r_max;
  for (int q = lane; q < 16 * nJ; q += EIG_NT) {
    const int js = q >> 4, a = (q >> 2) & 3, b = q & 3;
    const size_t row = (size_t)atom * (4 * JMAX) + 4 * js + a;
    double s = 0.0;
    if (g.vj_fp32) {
      const float* vr = (const float*)g.vj + row * vld;
      for (int m = 0; m < d; ++m) s += (double)vr[m] * x[4 * m + b];
    } else {
      const double* vr = (const double*)g.vj + row * vld;
      for (int m = 0; m < d; ++m) s += vr[m] * x[4 * m + b];
    }
    g.rho[(size_t)(p0 + js) * 16 + a * 4 + b] = s;
  }
}

size_t eig_lds_bytes(int r_max) { return (size_t)4 * r_max * (LB + 4) * sizeof(double); }
size_t rho_lds_bytes(int r_max) { return (size_t)4 * r_max * 4 * sizeof(double); }

void launch_eig(const EigArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_eig, dim3(a.n_atoms), dim3(EIG_NT), eig_lds_bytes(a.r_max), st, a);
}
void launch_rho(const RhoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_rho, dim3(a.n_atoms), dim3(EIG_NT), rho_lds_bytes(a.r_max), st, a);
}

}  // namespace tbk
