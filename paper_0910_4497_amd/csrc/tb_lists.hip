// Neighbour lists, cutoff spheres, Slater-Koster pair data and the local
// coupling structure of every sphere (Sec. 2: locality; Eq. 1: Hamiltonian).
//
//   k_cell_*     cell lists: on each periodic axis the box is cut into
//                cells no shorter than the cluster radius (at most 64), a
//                non-periodic axis is one cell; atoms are binned by counting
//                (count, scan, scatter).
//   k_lists      one workgroup per atom: the candidates of the 27 (fewer
//                when an axis has fewer than 3 cells) neighbouring cells,
//                hop list and cutoff sphere by minimum image, each put in
//                index order by rank (the sphere after its target).
//   k_union      grouped form (Sec. 3: the m atoms of a group share one
//                Hamiltonian): one workgroup per group of consecutive atoms;
//                the union of the members' spheres (sort + unique in LDS)
//                replaces each member's sphere, the member first.
//   k_pairs      per ordered pair: direction cosines h = d/|d| and the hopping
//                scale s(|d|) (FP64 and FP32 copies), and the reverse slot.
//   k_local      one workgroup per sphere: local couplings (a -> b, slot) with
//                the cluster-frame rule |x_b - x_a| < rm, x = position
//                relative to the target; Frobenius norm of the local H; the
//                local indices of the rho row atoms J = {i} + hop(i).
//   k_rowptr     prefix sum of 1 + |hop(i)| (rho pair layout); k_colj fills
//                the pair columns, one thread per entry.
#include "tb_internal.h"

namespace tbk {

constexpr int LIST_NT = 256;

__device__ __forceinline__ void stat_max(int64_t* stats, int slot, int64_t v) {
  atomicMax((unsigned long long*)&stats[slot], (unsigned long long)v);
}
__device__ __forceinline__ void stat_flag(int64_t* stats, int64_t bits) {
  atomicOr((unsigned long long*)&stats[ST_FLAGS], (unsigned long long)bits);
}

// Inclusive scan of one value per thread over a LIST_NT-thread workgroup
// (shuffles within each wave, then the wave totals); every thread also gets
// the workgroup total. s_w: LIST_NT / 64 entries of shared memory.
template <typename T>
__device__ __forceinline__ T block_scan(T v, T* s_w, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) s_w[wave] = v;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < LIST_NT / 64; ++w) {
    const T x = s_w[w];
    pre += w < wave ? x : 0;
    tot += x;
  }
  __syncthreads();                                   // s_w is reused by the next call
  total = tot;
  return v + pre;
}

__global__ void k_cell_zero(int* __restrict__ cnt, int m) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < m; q += gridDim.x * blockDim.x) cnt[q] = 0;
}

__device__ __forceinline__ int cell_coord(double x, const Box& box, const CellGrid& cg, int a) {
  if (cg.n[a] == 1) return 0;
  double w = x - box.L[a] * floor(x / box.L[a]);          // into [0, L)
  if (!(w >= 0.0)) w = 0.0;                               // non-finite: flagged by k_lists
  int c = (int)(w / cg.len[a]);
  return c < 0 ? 0 : (c >= cg.n[a] ? cg.n[a] - 1 : c);
}

__global__ void k_cell_count(int n, const double* __restrict__ pos, Box box, CellGrid cg,
                             int* __restrict__ cell_of, int* __restrict__ cell_cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = cell_coord(pos[3 * i], box, cg, 0), c1 = cell_coord(pos[3 * i + 1], box, cg, 1),
            c2 = cell_coord(pos[3 * i + 2], box, cg, 2);
  const int id = (c0 * cg.n[1] + c1) * cg.n[2] + c2;
  cell_of[i] = id;
  atomicAdd(&cell_cnt[id], 1);
}

// single workgroup: exclusive scan of the counts into cell_start[0..m], and
// the counts reset to serve as scatter cursors
__global__ void __launch_bounds__(LIST_NT) k_cell_scan(int m, int* __restrict__ cell_cnt,
                                                       int* __restrict__ cell_start) {
  __shared__ int s_w[LIST_NT / 64];
  const int tid = threadIdx.x;
  int base = 0;                                      // the same in every thread
  for (int b0 = 0; b0 < m; b0 += LIST_NT) {
    const int q = b0 + tid;
    const int v = q < m ? cell_cnt[q] : 0;
    int tot;
    const int incl = block_scan(v, s_w, tot);
    if (q < m) {
      cell_start[q] = base + incl - v;
      cell_cnt[q] = base + incl - v;
    }
    base += tot;
  }
  if (tid == 0) cell_start[m] = base;
}

__global__ void k_cell_fill(int n, const int* __restrict__ cell_of, int* __restrict__ cursor,
                            int* __restrict__ cell_atoms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cell_atoms[atomicAdd(&cursor[cell_of[i]], 1)] = i;
}

// Dynamic LDS: s_cj [nc_max] sphere members (unsorted, target excluded).
__global__ void __launch_bounds__(LIST_NT)
k_lists(int n, const double* __restrict__ pos, Box box, CellGrid cg, const int* __restrict__ cell_of,
        const int* __restrict__ cell_start, const int* __restrict__ cell_atoms, double r_list,
        double r_cluster, int nc_max, int zmax, int* __restrict__ hop_n, int* __restrict__ hop_j,
        double* __restrict__ hop_d, int* __restrict__ clu_n, int* __restrict__ clu_j, int64_t* stats) {
  extern __shared__ int s_cj[];
  __shared__ int s_hj[ZMAX_CAP];
  __shared__ double s_hd[ZMAX_CAP][4];
  __shared__ int s_nh, s_nc;
  __shared__ int s_cb[27], s_co[28];            // scanned cells: first candidate, range offsets
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) { s_nh = 0; s_nc = 0; }
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  const double rl2 = r_list * r_list, rc2 = r_cluster * r_cluster;
  bool nonfinite = !(isfinite(xi) && isfinite(yi) && isfinite(zi));
  // the cells to scan on each axis: the atom's and its two neighbours, or
  // every cell when the axis has fewer than three
  const int ci = cell_of[i];
  const int cc[3] = {ci / (cg.n[1] * cg.n[2]), (ci / cg.n[2]) % cg.n[1], ci % cg.n[2]};
  int lo[3], cnt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (cg.n[a] >= 3) { lo[a] = cc[a] - 1; cnt[a] = 3; }
    else { lo[a] = 0; cnt[a] = cg.n[a]; }
  }
  // The candidates of all scanned cells form one flat range: the first
  // threads read the cells' bounds (one round trip), wave 0 scans their
  // sizes, and every thread then takes candidates q = tid, tid + LIST_NT, ...
  // of the range in batches whose loads are all issued before the distances
  // are formed (two round trips per batch instead of three per cell). The
  // hop and sphere members are put in index order below, so the order in
  // which they are found does not matter.
  const int ncs = cnt[0] * cnt[1] * cnt[2];     // <= 27 distinct cells
  if (tid < ncs) {
    const int u0 = tid / (cnt[1] * cnt[2]), u1 = (tid / cnt[2]) % cnt[1], u2 = tid % cnt[2];
    const int a0 = (lo[0] + u0 + cg.n[0]) % cg.n[0], a1 = (lo[1] + u1 + cg.n[1]) % cg.n[1],
              a2 = (lo[2] + u2 + cg.n[2]) % cg.n[2];
    const int cell = (a0 * cg.n[1] + a1) * cg.n[2] + a2;
    const int b0 = cell_start[cell];
    s_cb[tid] = b0;
    s_co[tid + 1] = cell_start[cell + 1] - b0;
  }
  __syncthreads();
  if (tid < 64) {                               // inclusive scan of the sizes, one wave
    int v = tid < ncs ? s_co[tid + 1] : 0;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int u = __shfl_up(v, off, 64);
      if (tid >= off) v += u;
    }
    if (tid < ncs) s_co[tid + 1] = v;
    if (tid == 0) s_co[0] = 0;
  }
  __syncthreads();
  const int total = s_co[ncs];
  constexpr int LB = 4;                         // candidates per thread and batch
  for (int q0 = tid; q0 < total; q0 += LB * LIST_NT) {
    int jj[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int q = q0 + u * LIST_NT;
      jj[u] = -1;
      if (q < total) {
        int c = 0, hi = ncs - 1;                // the last cell whose range starts at or before q
        while (c < hi) {
          const int mid = (c + hi + 1) >> 1;
          if (s_co[mid] <= q) c = mid; else hi = mid - 1;
        }
        jj[u] = cell_atoms[s_cb[c] + (q - s_co[c])];
      }
    }
    double px[LB], py[LB], pz[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int j = jj[u] < 0 ? i : jj[u];
      px[u] = pos[3 * j]; py[u] = pos[3 * j + 1]; pz[u] = pos[3 * j + 2];
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int j = jj[u];
      if (j < 0 || j == i) continue;
      const double dx = mic(px[u] - xi, box.L[0], box.per[0]);
      const double dy = mic(py[u] - yi, box.L[1], box.per[1]);
      const double dz = mic(pz[u] - zi, box.L[2], box.per[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (!isfinite(r2)) nonfinite = true;
      if (r2 < rl2) {
        const int slot = atomicAdd(&s_nh, 1);
        if (slot < zmax) { s_hj[slot] = j; s_hd[slot][0] = dx; s_hd[slot][1] = dy; s_hd[slot][2] = dz; s_hd[slot][3] = sqrt(r2); }
      }
      if (r2 < rc2) {
        const int slot = atomicAdd(&s_nc, 1);
        if (slot < nc_max - 1) s_cj[slot] = j;
      }
    }
  }
  __syncthreads();
  const int nh = s_nh, ncl = s_nc + 1;          // the sphere counts its target
  const int mh = nh < zmax ? nh : zmax, mc = ncl - 1 < nc_max - 1 ? ncl - 1 : nc_max - 1;
  // index order by rank (the members are distinct)
  if (tid < mh) {
    const int j = s_hj[tid];
    int rank = 0;
    for (int e = 0; e < mh; ++e) rank += s_hj[e] < j;
    const int64_t q = (int64_t)i * zmax + rank;
    hop_j[q] = j;
    hop_d[4 * q] = s_hd[tid][0]; hop_d[4 * q + 1] = s_hd[tid][1];
    hop_d[4 * q + 2] = s_hd[tid][2]; hop_d[4 * q + 3] = s_hd[tid][3];
  }
  for (int t = tid; t < mc; t += LIST_NT) {
    const int j = s_cj[t];
    int rank = 0;
    for (int e = 0; e < mc; ++e) rank += s_cj[e] < j;
    clu_j[(int64_t)i * nc_max + 1 + rank] = j;
  }
  if (nonfinite) stat_flag(stats, FL_NONFINITE);
  if (tid == 0) {
    clu_j[(int64_t)i * nc_max] = i;
    if (nh > zmax) stat_flag(stats, FL_HOP_OVERFLOW);
    if (ncl > nc_max) stat_flag(stats, FL_CLUSTER_OVERFLOW);
    hop_n[i] = mh;
    clu_n[i] = mc + 1;
    stat_max(stats, ST_MAX_HOP, nh);
    stat_max(stats, ST_MAX_CLUSTER, ncl);
  }
}

// Dynamic LDS: s_v [pcap] (a power of two >= m * nc_max). Every read of the
// members' spheres ends before the first barrier, and the groups own disjoint
// rows, so the spheres are rewritten in place.
__global__ void __launch_bounds__(LIST_NT)
k_union(int n, int m, const double* __restrict__ pos, Box box, double r_cluster, int nc_max,
        int* __restrict__ clu_n, int* __restrict__ clu_j, int64_t* stats) {
  extern __shared__ int s_v[];
  __shared__ int s_off[GROUP_MAX + 1];
  __shared__ int s_pos[GROUP_MAX];          // rank of each member in the union
  __shared__ int s_part[LIST_NT];
  const int tid = threadIdx.x;
  const int g0 = blockIdx.x * m;
  const int mm = n - g0 < m ? n - g0 : m;
  if (tid == 0) {
    int o = 0;
    for (int k = 0; k < mm; ++k) { s_off[k] = o; o += clu_n[g0 + k]; }
    s_off[mm] = o;
  }
  __syncthreads();
  const int tot = s_off[mm];
  int P = 1;
  while (P < tot) P <<= 1;
  for (int k = 0; k < mm; ++k) {
    const int nk = s_off[k + 1] - s_off[k];
    for (int t = tid; t < nk; t += LIST_NT) s_v[s_off[k] + t] = clu_j[(int64_t)(g0 + k) * nc_max + t];
  }
  for (int t = tot + tid; t < P; t += LIST_NT) s_v[t] = INT_MAX;
  // images: the union is taken in the frame of each member, which is
  // unambiguous while |(d_ik)_a| + r_cluster < L_a / 2 for all members i, k
  for (int q = tid; q < mm * mm; q += LIST_NT) {
    const int i = g0 + q / mm, k = g0 + q % mm;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (box.per[a] && !(fabs(mic(pos[3 * k + a] - pos[3 * i + a], box.L[a], 1)) + r_cluster < 0.5 * box.L[a]))
        stat_flag(stats, FL_GROUP_IMAGE);
  }
  __syncthreads();
  // bitonic sort, ascending
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P / 2; t += LIST_NT) {
        const int lo = 2 * stride * (t / stride) + t % stride, hi = lo + stride;
        const int a = s_v[lo], b = s_v[hi];
        if ((a > b) == ((lo & size) == 0)) { s_v[lo] = b; s_v[hi] = a; }
      }
      __syncthreads();
    }
  // unique values: first of each run; chunked exclusive scan of their count
  const int C = (tot + LIST_NT - 1) / LIST_NT;
  const int t0 = tid * C, t1 = t0 + C < tot ? t0 + C : tot;
  int cnt = 0;
  for (int t = t0; t < t1; ++t) cnt += (t == 0 || s_v[t] != s_v[t - 1]);
  s_part[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < LIST_NT; off <<= 1) {
    const int add = tid >= off ? s_part[tid - off] : 0;
    __syncthreads();
    s_part[tid] += add;
    __syncthreads();
  }
  const int u = s_part[LIST_NT - 1];
  int p = s_part[tid] - cnt;
  for (int t = t0; t < t1; ++t) {
    if (!(t == 0 || s_v[t] != s_v[t - 1])) continue;
    const int v = s_v[t] - g0;
    if (v >= 0 && v < mm) s_pos[v] = p;
    ++p;
  }
  __syncthreads();
  // member i: slot 0 = i, then the union without i, in index order
  p = s_part[tid] - cnt;
  for (int t = t0; t < t1; ++t) {
    if (!(t == 0 || s_v[t] != s_v[t - 1])) continue;
    const int v = s_v[t];
    for (int k = 0; k < mm; ++k) {
      const int pi = s_pos[k];
      if (p == pi) continue;
      const int slot = p < pi ? p + 1 : p;
      if (slot < nc_max) clu_j[(int64_t)(g0 + k) * nc_max + slot] = v;
    }
    ++p;
  }
  if (tid < mm) {
    clu_j[(int64_t)(g0 + tid) * nc_max] = g0 + tid;
    clu_n[g0 + tid] = u < nc_max ? u : nc_max;
  }
  if (tid == 0) {
    if (u > nc_max) stat_flag(stats, FL_CLUSTER_OVERFLOW);
    stat_max(stats, ST_MAX_CLUSTER, u);
  }
}

__global__ void k_pairs(int n, int zmax, Model M, const int* __restrict__ hop_n, const int* __restrict__ hop_j,
                        const double* __restrict__ hop_d, double* __restrict__ pair64,
                        float* __restrict__ pair32, int* __restrict__ hop_rev) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * zmax) return;
  const int i = (int)(q / zmax), slot = (int)(q % zmax);
  double hx = 0, hy = 0, hz = 0, s = 0;
  int rev = -1;
  if (slot < hop_n[i]) {
    const double r = hop_d[4 * q + 3];
    hx = hop_d[4 * q] / r; hy = hop_d[4 * q + 1] / r; hz = hop_d[4 * q + 2] / r;
    double ds;
    hop_scale(M, r, s, ds);
    const int j = hop_j[q];
    const int nj = hop_n[j];
    for (int t = 0; t < nj; ++t)
      if (hop_j[(int64_t)j * zmax + t] == i) { rev = t; break; }
  }
  pair64[4 * q] = hx; pair64[4 * q + 1] = hy; pair64[4 * q + 2] = hz; pair64[4 * q + 3] = s;
  pair32[4 * q] = (float)hx; pair32[4 * q + 1] = (float)hy; pair32[4 * q + 2] = (float)hz;
  pair32[4 * q + 3] = (float)s;
  hop_rev[q] = rev;
}

// Local index of global atom g in the sphere list c (c[0] = target, c[1..n-1]
// sorted increasingly), or -1.
__device__ __forceinline__ int find_local(const int* c, int n, int g) {
  if (g == c[0]) return 0;
  int lo = 1, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = c[mid];
    if (v == g) return mid;
    if (v < g) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// 64 VGPRs: eight workgroups per compute unit, so that one round of
// workgroups covers 2048 spheres
__global__ void __launch_bounds__(LIST_NT, 8)
k_local(int n_atoms, Model M, const double* __restrict__ pos, Box box, int nc_max, int zmax, int64_t emax,
        const int* __restrict__ hop_n, const int* __restrict__ hop_j, const double* __restrict__ hop_d,
        const double* __restrict__ pair64, const int* __restrict__ clu_n, const int* __restrict__ clu_j,
        int* __restrict__ loc_off, uint32_t* __restrict__ loc_ent, double* __restrict__ hnorm,
        int* __restrict__ jloc, int64_t* stats, int cache_b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int n = clu_n[i];
  int* s_c = (int*)smem;                               // [nc_max]
  int* s_cnt = s_c + nc_max;                           // [nc_max + 1]
  // [nc_max][3], 8-byte aligned; addressed from smem by a byte offset so that
  // its accesses stay LDS accesses (not flat ones)
  double* s_x = (double*)(smem + ((((size_t)(2 * nc_max + 2) * sizeof(int)) + 7) & ~(size_t)7));
  // [nc_max][zmax] local partner of each hop slot, or -1 (cache_b: short hop
  // lists whose table fits the LDS budget; else pass 2 repeats the tests)
  int16_t* s_b = (int16_t*)(s_x + 3 * (size_t)nc_max);
  __shared__ double s_red[LIST_NT / 64];
  __shared__ int s_wsum[LIST_NT / 64];
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  for (int a = tid; a < n; a += LIST_NT) {
    const int g = clu_j[(int64_t)i * nc_max + a];
    s_c[a] = g;
    s_x[3 * a] = mic(pos[3 * g] - xi, box.L[0], box.per[0]);
    s_x[3 * a + 1] = mic(pos[3 * g + 1] - yi, box.L[1], box.per[1]);
    s_x[3 * a + 2] = mic(pos[3 * g + 2] - zi, box.L[2], box.per[2]);
  }
  __syncthreads();
  const double rm2 = M.rm * M.rm;
  const double kfro = M.v_sss * M.v_sss + 2 * M.v_sps * M.v_sps + M.v_pps * M.v_pps + 2 * M.v_ppp * M.v_ppp;
  double fro = 0.0;
  // the coupling rule: hop pair (g -> hop slot t) of local atom a couples a
  // to local atom b when both lie in the sphere and |x_b - x_a| < rm
  auto coupling = [&](int a, int g, int t, int& b) -> bool {
    const int64_t q = (int64_t)g * zmax + t;
    if (hop_d[4 * q + 3] >= M.rm) return false;
    b = find_local(s_c, n, hop_j[q]);
    if (b < 0) return false;
    const double ex = s_x[3 * b] - s_x[3 * a], ey = s_x[3 * b + 1] - s_x[3 * a + 1],
                 ez = s_x[3 * b + 2] - s_x[3 * a + 2];
    return ex * ex + ey * ey + ez * ez < rm2;             // else it wraps behind the target
  };
  // long hop lists (zmax > 32): a wave per local atom, lanes over its hop
  // slots; short ones: a thread per local atom
  const bool by_wave = zmax > 32;
  const int lane = tid & 63, wave = tid >> 6;
  // pass 1: count couplings per local atom
  if (by_wave) {
    for (int a = wave; a < n; a += LIST_NT / 64) {
      const int g = s_c[a];
      const int nh = hop_n[g];
      int cnt = 0;
      if (lane == 0) fro += M.eps_s * M.eps_s + 3 * M.eps_p * M.eps_p;
      for (int t = lane; t < nh; t += 64) {
        int b;
        if (!coupling(a, g, t, b)) continue;
        ++cnt;
        const double sv = pair64[4 * ((int64_t)g * zmax + t) + 3];
        fro += kfro * sv * sv;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
      if (lane == 0) s_cnt[a + 1] = cnt;
    }
  } else {
    // the slots' distance, partner and hopping scale are loaded a batch at
    // a time, all before they are used; the local partner (or -1) of every
    // slot is kept for pass 2
    constexpr int SB = 6;
    for (int a = tid; a < n; a += LIST_NT) {
      const int g = s_c[a];
      const int nh = hop_n[g];
      int cnt = 0;
      fro += M.eps_s * M.eps_s + 3 * M.eps_p * M.eps_p;
      for (int t0 = 0; t0 < nh; t0 += SB) {
        double dd[SB], sv[SB];
        int hj[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int64_t q = (int64_t)g * zmax + (t0 + u < nh ? t0 + u : t0);
          dd[u] = hop_d[4 * q + 3]; hj[u] = hop_j[q]; sv[u] = pair64[4 * q + 3];
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
          const int t = t0 + u;
          if (t >= nh) break;
          int b = -1;
          if (dd[u] < M.rm) {
            b = find_local(s_c, n, hj[u]);
            if (b >= 0) {
              const double ex = s_x[3 * b] - s_x[3 * a], ey = s_x[3 * b + 1] - s_x[3 * a + 1],
                           ez = s_x[3 * b + 2] - s_x[3 * a + 2];
              if (!(ex * ex + ey * ey + ez * ez < rm2)) b = -1;   // it wraps behind the target
            }
          }
          if (cache_b) s_b[a * zmax + t] = (int16_t)b;
          if (b < 0) continue;
          ++cnt;
          fro += kfro * sv[u] * sv[u];
        }
      }
      s_cnt[a + 1] = cnt;
    }
  }
  if (tid == 0) s_cnt[0] = 0;
  fro = wave_sum(fro);
  if ((tid & 63) == 0) s_red[tid >> 6] = fro;
  __syncthreads();
  // offsets: inclusive scan of s_cnt[1..n], each thread over a contiguous
  // chunk, the chunk totals scanned across the workgroup
  {
    const int ch = (n + LIST_NT - 1) / LIST_NT;
    const int a0 = 1 + tid * ch, a1 = a0 + ch < n + 1 ? a0 + ch : n + 1;
    int tot = 0;
    for (int a = a0; a < a1; ++a) tot += s_cnt[a];
    int v = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    if (lane == 63) s_wsum[wave] = v;
    __syncthreads();
    int run = v - tot;                                 // exclusive within the wave
    for (int w = 0; w < wave; ++w) run += s_wsum[w];
    for (int a = a0; a < a1; ++a) { run += s_cnt[a]; s_cnt[a] = run; }
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int w = 0; w < LIST_NT / 64; ++w) f += s_red[w];
    hnorm[i] = sqrt(f);
    if (s_cnt[n] > emax) stat_flag(stats, FL_COUPLING_OVERFLOW);
    stat_max(stats, ST_MAX_COUPLINGS, s_cnt[n]);
  }
  __syncthreads();
  for (int a = tid; a <= n; a += LIST_NT) loc_off[(int64_t)i * (nc_max + 1) + a] = s_cnt[a];
  // pass 2: write couplings (b | slot << LOCAL_BITS) in hop-list order
  if (by_wave) {
    for (int a = wave; a < n; a += LIST_NT / 64) {
      const int g = s_c[a];
      const int nh = hop_n[g];
      int64_t base = s_cnt[a];
      for (int t0 = 0; t0 < nh; t0 += 64) {
        const int t = t0 + lane;
        int b = 0;
        const bool ok = t < nh && coupling(a, g, t, b);
        const uint64_t m = __ballot(ok);
        const int64_t e = base + __popcll(m & ((1ull << lane) - 1ull));
        if (ok && e < emax) loc_ent[(int64_t)i * emax + e] = (uint32_t)b | ((uint32_t)t << LOCAL_BITS);
        base += __popcll(m);
      }
    }
  } else {
    for (int a = tid; a < n; a += LIST_NT) {
      const int g = s_c[a];
      const int nh = hop_n[g];
      int64_t e = s_cnt[a];
      for (int t = 0; t < nh; ++t) {
        int b;
        if (cache_b) b = s_b[a * zmax + t];
        else if (!coupling(a, g, t, b)) b = -1;
        if (b < 0) continue;
        if (e < emax) loc_ent[(int64_t)i * emax + e] = (uint32_t)b | ((uint32_t)t << LOCAL_BITS);
        ++e;
      }
    }
  }
  // rho row atoms: J[0] = target (local 0), then hop(i) in list order
  {
    int* jl = jloc + (int64_t)i * (zmax + 1);
    const int nh = hop_n[i];
    for (int t = tid; t < zmax + 1; t += LIST_NT)
      jl[t] = t == 0 ? 0 : (t <= nh ? find_local(s_c, n, hop_j[(int64_t)i * zmax + t - 1]) : -1);
  }
}

__global__ void __launch_bounds__(LIST_NT) k_rowptr(int n, const int* __restrict__ hop_n,
                                                    int64_t* __restrict__ row_ptr) {
  // single workgroup: chunks of LIST_NT rows, each a workgroup scan
  __shared__ int64_t s_w[LIST_NT / 64];
  const int tid = threadIdx.x;
  if (tid == 0) row_ptr[0] = 0;
  int64_t base = 0;                                  // the same in every thread
  for (int b0 = 0; b0 < n; b0 += LIST_NT) {
    const int i = b0 + tid;
    const int64_t v = (i < n) ? 1 + hop_n[i] : 0;
    int64_t tot;
    const int64_t incl = block_scan(v, s_w, tot);
    if (i < n) row_ptr[i + 1] = base + incl;
    base += tot;
  }
}

// rho pair layout: row i lists the target i, then its hop list (one thread
// per entry, after the scan of k_rowptr)
__global__ void k_colj(int n, int zmax, const int* __restrict__ hop_n, const int* __restrict__ hop_j,
                       const int64_t* __restrict__ row_ptr, int* __restrict__ col_j) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * (zmax + 1)) return;
  const int i = (int)(q / (zmax + 1)), t = (int)(q % (zmax + 1));
  if (t > hop_n[i]) return;
  col_j[row_ptr[i] + t] = t == 0 ? i : hop_j[(int64_t)i * zmax + t - 1];
}

void launch_build(tb_ctx* c, const double* pos, double r_list, hipStream_t st) {
  const int n = (int)c->n_atoms;
  // cells no shorter than the cluster radius on periodic axes (so a sphere
  // lies in the 3 x 3 x 3 cells around its target); one cell otherwise
  CellGrid cg;
  for (int a = 0; a < 3; ++a) {
    int m = c->box.per[a] ? (int)floor(c->box.L[a] / c->r_cluster) : 1;
    m = m < 1 ? 1 : (m > NCELL_AXIS_MAX ? NCELL_AXIS_MAX : m);
    cg.n[a] = m;
    cg.len[a] = c->box.L[a] / m;
  }
  const int ncell = cg.n[0] * cg.n[1] * cg.n[2];
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_cell_zero, dim3((ncell + 255) / 256), dim3(256), 0, st, c->cell_cnt, ncell);
  hipLaunchKernelGGL(k_cell_count, dim3(nb), dim3(256), 0, st, n, pos, c->box, cg, c->cell_of, c->cell_cnt);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(LIST_NT), 0, st, ncell, c->cell_cnt, c->cell_start);
  hipLaunchKernelGGL(k_cell_fill, dim3(nb), dim3(256), 0, st, n, c->cell_of, c->cell_cnt, c->cell_atoms);
  hipLaunchKernelGGL(k_lists, dim3(n), dim3(LIST_NT), (size_t)c->nc_max * sizeof(int), st, n, pos, c->box, cg,
                     c->cell_of, c->cell_start, c->cell_atoms, r_list, c->r_cluster, c->nc_max, c->zmax, c->hop_n,
                     c->hop_j, c->hop_d, c->clu_n, c->clu_j, c->stats);
  if (c->group_m > 1) {
    int pcap = 1;
    while (pcap < c->group_m * c->nc_max) pcap <<= 1;
    hipLaunchKernelGGL(k_union, dim3((n + c->group_m - 1) / c->group_m), dim3(LIST_NT), (size_t)pcap * sizeof(int),
                       st, n, c->group_m, pos, c->box, c->r_cluster, c->nc_max, c->clu_n, c->clu_j, c->stats);
  }
  const int64_t np = (int64_t)n * c->zmax;
  hipLaunchKernelGGL(k_pairs, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, n, c->zmax, c->model, c->hop_n,
                     c->hop_j, c->hop_d, c->pair64, c->pair32, c->hop_rev);
  const size_t lds_base = (size_t)c->nc_max * (4 + 4 + 24) + 64;
  const size_t lds_b = (size_t)c->nc_max * c->zmax * sizeof(int16_t);
  const int cache_b = c->zmax <= 32 && lds_base + lds_b <= 48 * 1024;
  const size_t lds_local = lds_base + (cache_b ? lds_b : 0);
  hipLaunchKernelGGL(k_local, dim3(n), dim3(LIST_NT), lds_local, st, n, c->model, pos, c->box, c->nc_max,
                     c->zmax, c->emax, c->hop_n, c->hop_j, c->hop_d, c->pair64, c->clu_n, c->clu_j, c->loc_off,
                     c->loc_ent, c->hnorm, c->jloc, c->stats, cache_b);
  hipLaunchKernelGGL(k_rowptr, dim3(1), dim3(LIST_NT), 0, st, n, c->hop_n, c->row_ptr);
  const int64_t nq = (int64_t)n * (c->zmax + 1);
  hipLaunchKernelGGL(k_colj, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, n, c->zmax, c->hop_n, c->hop_j,
                     c->row_ptr, c->col_j);
}

}  // namespace tbk
