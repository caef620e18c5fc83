// C-ABI of libtbkrylov: argument validation, work-buffer ownership and the
// launch sequence of the kernels. See include/tbkrylov.h for the contract.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include <float.h>

#include "tb_internal.h"

namespace tbk {
__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
__global__ void k_zero_i64(int64_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace tbk

using namespace tbk;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(TB_EHIP, "%s: %s", #expr, hipGetErrorString(_e));   \
  } while (0)

static const int MU_ITERS = 13;   // multisection steps (5 bits each)

// phase timing: returns the slot of the start event, or -1 when disabled/full
static int prof_begin(tb_ctx* c, int phase) {
  if (!c->prof) return -1;
  if (c->ev_used >= PROF_MAX) { ++c->ev_dropped; return -1; }
  const int k = c->ev_used++;
  c->ev_phase[k] = phase;
  hipEventRecord(c->ev_pool[2 * k], c->stream);
  return k;
}
static void prof_end(tb_ctx* c, int k) {
  if (k >= 0) hipEventRecord(c->ev_pool[2 * k + 1], c->stream);
}

extern "C" const char* tb_last_error(void) { return g_err.c_str(); }

template <typename T>
static hipError_t alloc(tb_ctx* c, T** p, size_t count) {
  const size_t b = count * sizeof(T) > 0 ? count * sizeof(T) : 16;
  c->bytes += b;
  return hipMalloc((void**)p, b);
}

extern "C" int tb_destroy(tb_ctx* c) {
  if (!c) return TB_OK;
  int dev_prev = 0;
  hipGetDevice(&dev_prev);
  hipSetDevice(c->device);
  void* ptrs[] = {c->hop_n, c->hop_j, c->hop_rev, c->hop_d, c->pair64, c->pair32, c->clu_n, c->clu_j,
                  c->loc_off, c->loc_ent, c->hnorm, c->jloc, c->row_ptr, c->col_j, c->vbuf, c->tab,
                  c->kused, c->vj, c->work_counter, c->lam, c->wgt, c->y1, c->ref_v, c->ref_p,
                  c->ref_n, c->seg, c->seg_n, c->evec, c->tri, c->eig_scratch, c->omega, c->mu_state, c->partial, c->xrep, c->eparts, c->stats,
                  c->cell_of, c->cell_atoms, c->cell_cnt, c->cell_start, c->wpart, c->virial, c->vsc};
  for (void* p : ptrs)
    if (p) hipFree(p);
  if (c->ev_pool) {
    for (int k = 0; k < 2 * PROF_MAX; ++k) hipEventDestroy(c->ev_pool[k]);
    delete[] c->ev_pool;
    delete[] c->ev_phase;
  }
  hipSetDevice(dev_prev);
  delete c;
  return TB_OK;
}

extern "C" int tb_create(tb_ctx** out, int hip_device, void* hip_stream, int64_t n_atoms_max,
                         int n_cluster_max, int r_max) {
  return tb_create_ex(out, hip_device, hip_stream, n_atoms_max, n_cluster_max, r_max, ZMAX_DEFAULT);
}

extern "C" int tb_create_ex(tb_ctx** out, int hip_device, void* hip_stream, int64_t n_atoms_max,
                            int n_cluster_max, int r_max, int hop_max) {
  if (!out) return fail(TB_EINVAL, "ctx pointer is null");
  *out = nullptr;
  if (hop_max < 1 || hop_max > ZMAX_CAP) return fail(TB_EINVAL, "hop_max must be in [1, %d]", ZMAX_CAP);
  if (n_atoms_max < 1 || n_atoms_max > (1 << 24)) return fail(TB_EINVAL, "n_atoms_max out of range");
  if (n_cluster_max < 1 || n_cluster_max > NCLUSTER_LIMIT)
    return fail(TB_EINVAL, "n_cluster_max must be in [1, %d]", NCLUSTER_LIMIT);
  if (r_max < 1 || r_max > RMAX_LIMIT) return fail(TB_EINVAL, "r_max must be in [1, %d]", RMAX_LIMIT);
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) return fail(TB_EINVAL, "hip_device %d not present", hip_device);
  HIP_TRY(hipSetDevice(hip_device));
  tb_ctx* c = new tb_ctx();
  memset((void*)c, 0, sizeof(tb_ctx));
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  c->na_max = n_atoms_max;
  c->nc_max = n_cluster_max;
  c->r_max = r_max;
  c->zmax = hop_max;
  c->emax = (int64_t)n_cluster_max * hop_max;
  const int64_t dmax = 4 * (int64_t)r_max;
  // band -> tridiagonal: reflectors of length 4, about d^2 / 8 of them
  c->ref_max = band_reflectors((int)dmax);

  // persistent Krylov workgroups: as many as fit on the device at once
  const size_t lds = lanczos_lds_bytes(n_cluster_max, r_max, false, 512, false, false, false);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  if (lds + LDS_RESERVE > LDS_CU) {
    delete c;
    return fail(TB_ECAPACITY, "n_cluster_max=%d, r_max=%d need %zu B of LDS per workgroup", n_cluster_max,
                r_max, lds);
  }
  hipError_t e = lanczos_set_lds(LDS_CU - LDS_RESERVE);
  if (e != hipSuccess) {
    delete c;
    return fail(TB_ECAPACITY, "LDS request of %zu B refused: %s", (size_t)(LDS_CU - LDS_RESERVE),
                hipGetErrorString(e));
  }
  e = static_scratch_init(hip_device);                 // tb_energy_forces_static's workspace address
  if (e != hipSuccess) {
    delete c;
    return fail(TB_EHIP, "address of the fixed device workspace: %s", hipGetErrorString(e));
  }
  e = eig_set_lds(r_max);
  if (e != hipSuccess || rho_lds_bytes(r_max) > LDS_CU) {
    delete c;
    return fail(TB_ECAPACITY, "r_max=%d too large for the eigensolver LDS: %s", r_max, hipGetErrorString(e));
  }
  c->n_cu = prop.multiProcessorCount;
  // default shape: 512 threads, workgroups per CU from the FP64 footprint
  // (at most 2), for both precisions; tb_autotune may change it
  int per_cu = (int)(LDS_CU / (lds + LDS_RESERVE));
  per_cu = per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu);
  for (int q = 0; q < 3; ++q) { c->lz_nt[q] = 512; c->lz_minw[q] = 4; c->lz_per_cu[q] = per_cu; c->lz_wide[q] = 0; }
  // workspace for the largest shape the tuner may pick: the smallest (FP32,
  // 256-thread) footprint, at most LZ_PER_CU_MAX per compute unit
  const size_t lds_min = lanczos_lds_bytes(n_cluster_max, r_max, true, 256, false, false, false);
  int pmax = (int)(LDS_CU / (lds_min + LDS_RESERVE));
  c->lz_per_cu_max = pmax < per_cu ? per_cu : (pmax > LZ_PER_CU_MAX ? LZ_PER_CU_MAX : pmax);
  c->eig_per_cu = eig_threads(r_max) <= 192 ? 6 : 4;
  int emx = (int)(LDS_CU / (eig_lds_bytes(r_max) + LDS_RESERVE));
  const int ewv = 2048 / eig_threads(r_max);            // 32 waves per CU
  emx = emx < ewv ? emx : ewv;
  emx = emx > EIG_PER_CU_MAX ? EIG_PER_CU_MAX : emx;
  c->eig_per_cu_max = emx < c->eig_per_cu ? c->eig_per_cu : emx;
  const int64_t n_wg_lz_max = (int64_t)c->n_cu * c->lz_per_cu_max < n_atoms_max
                                  ? (int64_t)c->n_cu * c->lz_per_cu_max : n_atoms_max;
  const int64_t n_wg_eig_max = (int64_t)c->n_cu * c->eig_per_cu_max < n_atoms_max
                                   ? (int64_t)c->n_cu * c->eig_per_cu_max : n_atoms_max;

  const int64_t N = n_atoms_max, NC = n_cluster_max, Z = hop_max;
  hipError_t a = hipSuccess;
#define ALLOC(ptr, cnt) \
  if (a == hipSuccess) a = alloc(c, &c->ptr, (size_t)(cnt));
  ALLOC(hop_n, N);
  ALLOC(hop_j, N * Z);
  ALLOC(hop_rev, N * Z);
  ALLOC(hop_d, N * Z * 4);
  ALLOC(pair64, N * Z * 4);
  ALLOC(pair32, N * Z * 4);
  ALLOC(cell_of, N);
  ALLOC(cell_atoms, N);
  ALLOC(cell_cnt, (int64_t)NCELL_AXIS_MAX * NCELL_AXIS_MAX * NCELL_AXIS_MAX);
  ALLOC(cell_start, (int64_t)NCELL_AXIS_MAX * NCELL_AXIS_MAX * NCELL_AXIS_MAX + 1);
  ALLOC(clu_n, N);
  ALLOC(clu_j, N * NC);
  ALLOC(loc_off, N * (NC + 1));
  ALLOC(loc_ent, N * c->emax);
  ALLOC(hnorm, N);
  ALLOC(jloc, N * (Z + 1));
  ALLOC(row_ptr, N + 1);
  ALLOC(col_j, N * (Z + 1));
  ALLOC(tab, N * r_max * 32);
  ALLOC(kused, N);
  ALLOC(work_counter, 16);
  ALLOC(lam, N * dmax);
  ALLOC(wgt, N * dmax);
  ALLOC(y1, N * 4 * dmax);
  ALLOC(ref_v, N * c->ref_max * 4);
  ALLOC(ref_p, N * c->ref_max);
  ALLOC(ref_n, N);
  c->seg_max = band_segments((int)dmax);
  ALLOC(seg, N * c->seg_max);
  ALLOC(seg_n, 2 * N);
  ALLOC(evec, N * dmax * dmax);
  ALLOC(vsc, N * dmax);
  ALLOC(tri, N * 2 * dmax);
  ALLOC(eig_scratch, n_wg_eig_max * dmax * 4 * eig_threads(r_max));
  ALLOC(mu_state, mu_state_doubles());
  ALLOC(partial, mu_partial_doubles());   // [region][blocks][points] of the mu reductions
  ALLOC(xrep, 2 * N);
  ALLOC(eparts, 8);
  ALLOC(wpart, ((N + 63) / 64) * 9);          // blocks of k_forces (64 atoms each)
  ALLOC(virial, 9);
  ALLOC(stats, ST_NSTATS);
#undef ALLOC
  if (a == hipSuccess) a = alloc(c, &c->omega, (size_t)n_wg_lz_max * 3 * r_max * 16);
  if (a == hipSuccess) {
    double* vb = nullptr;
    a = alloc(c, &vb, (size_t)n_wg_lz_max * r_max * 4 * NC * 4);
    c->vbuf = vb;
  }
  if (a == hipSuccess) {
    double* v = nullptr;
    a = alloc(c, &v, (size_t)N * 4 * (Z + 1) * dmax);
    c->vj = v;
  }
  if (a != hipSuccess) {
    tb_destroy(c);
    return fail(TB_EHIP, "work allocation of %zu B failed: %s", c->bytes, hipGetErrorString(a));
  }
  HIP_TRY(hipMemset(c->stats, 0, ST_NSTATS * sizeof(int64_t)));
  HIP_TRY(hipMemset(c->mu_state, 0, mu_state_doubles() * sizeof(double)));
  HIP_TRY(hipMemset(c->kused, 0, N * sizeof(int)));
  HIP_TRY(hipMemset(c->ref_n, 0, N * sizeof(int)));
  HIP_TRY(hipMemset(c->seg_n, 0, 2 * N * sizeof(int)));
  HIP_TRY(hipDeviceSynchronize());
  c->nnz_pairs = -1;
  *out = c;
  return TB_OK;
}

static bool finite_params(const tb_params* p) {
  const double* v = &p->eps_s;
  const int nd = (int)((sizeof(tb_params) - sizeof(int64_t)) / sizeof(double));
  for (int q = 0; q < nd; ++q)
    if (!isfinite(v[q])) return false;
  return true;
}

extern "C" int tb_build_local_H(tb_ctx* c, int64_t n_atoms, const double* pos, const double* cell_host,
                                const int* periodic_host, const tb_params* p, double r_cluster,
                                int* n_cluster_out) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (!pos || !cell_host || !periodic_host || !p) return fail(TB_EINVAL, "null argument");
  if (n_atoms < 1 || n_atoms > c->na_max)
    return fail(TB_ECAPACITY, "n_atoms=%lld outside [1, %lld]", (long long)n_atoms, (long long)c->na_max);
  if (p->struct_size != (int64_t)sizeof(tb_params))
    return fail(TB_EINVAL, "tb_params.struct_size=%lld, expected %zu", (long long)p->struct_size,
                sizeof(tb_params));
  if (!finite_params(p)) return fail(TB_EINVAL, "non-finite model parameter");
  if (!(p->r1 > 0 && p->rm > p->r1 && p->d1 > 0 && p->dm > p->d1 && p->rc > 0 && p->dc > 0))
    return fail(TB_EINVAL, "radial cutoffs must satisfy 0 < r1 < rm and 0 < d1 < dm");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (a != b && cell_host[3 * a + b] != 0.0)
        return fail(TB_EUNSUPPORTED, "only orthorhombic cells are supported");
  const double r_list = p->rm > p->dm ? p->rm : p->dm;
  if (!isfinite(r_cluster) || r_cluster <= r_list)
    return fail(TB_EINVAL, "r_cluster=%g must exceed the hopping/pair cutoff %g", r_cluster, r_list);
  Box box;
  for (int a = 0; a < 3; ++a) {
    box.per[a] = periodic_host[a] ? 1 : 0;
    box.L[a] = cell_host[4 * a];
    if (box.per[a]) {
      if (!(isfinite(box.L[a]) && box.L[a] > 0)) return fail(TB_EINVAL, "periodic box length %d invalid", a);
      if (r_cluster >= 0.5 * box.L[a])
        return fail(TB_ECUTOFF, "r_cluster=%g >= half the box length %g on axis %d", r_cluster, box.L[a], a);
    } else {
      box.L[a] = 1.0;
    }
  }
  HIP_TRY(hipSetDevice(c->device));
  Model M;
  memcpy(&M, &p->eps_s, sizeof(Model));
  c->model = M;
  c->box = box;
  c->r_cluster = r_cluster;
  c->n_atoms = n_atoms;
  const int n = (int)n_atoms;
  hipStream_t st = c->stream;
  const int pk = prof_begin(c, 0);
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, c->stats, ST_NSTATS);
  launch_build(c, pos, r_list, st);
  prof_end(c, pk);
  if (n_cluster_out) HIP_TRY(hipMemcpyAsync(n_cluster_out, c->clu_n, n * sizeof(int), hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipGetLastError());
  c->stage = 1;
  c->have_virial = 0;
  c->nnz_pairs = -1;
  return TB_OK;
}

// LDS residency of the Krylov kernel for a launch shape: the orthogonality
// estimates, then FP32 copies of A_j, B_j, then a second block buffer (V_{k-1}
// read from LDS), each taken while the footprint still lets `per_cu`
// workgroups share a compute unit. lds = 0 when even the base footprint does not.
struct LzPlan { int nt, minw, per_cu, n_wg; size_t lds; int om_lds, ab_lds, vprev_lds; };
static LzPlan lanczos_plan(const tb_ctx* c, bool fp32, int nt, int minw, int per_cu) {
  LzPlan p{nt, minw, per_cu, c->n_cu * per_cu, 0, 0, 0, 0};
  auto fits = [&](size_t l) { return (l + LDS_RESERVE) * per_cu <= LDS_CU; };
  const size_t l0 = lanczos_lds_bytes(c->nc_max, c->r_max, fp32, nt, false, false, false);
  const size_t l1 = lanczos_lds_bytes(c->nc_max, c->r_max, fp32, nt, true, false, false);
  const size_t l2 = lanczos_lds_bytes(c->nc_max, c->r_max, fp32, nt, true, true, false);
  const size_t l3 = lanczos_lds_bytes(c->nc_max, c->r_max, fp32, nt, true, true, true);
  if (!fits(l0) && per_cu > 1) return p;
  p.om_lds = fits(l1); p.ab_lds = p.om_lds && fits(l2); p.vprev_lds = p.ab_lds && fits(l3);
  p.lds = p.vprev_lds ? l3 : (p.ab_lds ? l2 : (p.om_lds ? l1 : l0));
  return p;
}

static LanczosArgs lanczos_args(const tb_ctx* c, int n, int r, const int* r_per_atom, int precision) {
  const bool fp32 = precision != TB_FP64;
  LanczosArgs la;
  la.atom0 = 0; la.n_atoms = n; la.r_default = r; la.r_per_atom = r_per_atom;
  la.clu_n = c->clu_n; la.clu_j = c->clu_j; la.loc_off = c->loc_off; la.loc_ent = c->loc_ent;
  la.zmax = c->zmax;
  la.hnorm = c->hnorm; la.jloc = c->jloc; la.hop_n = c->hop_n;
  la.pair = fp32 ? (const void*)c->pair32 : (const void*)c->pair64;
  la.nc_max = c->nc_max; la.emax = c->emax; la.r_max = c->r_max;
  la.eps_s = c->model.eps_s; la.eps_p = c->model.eps_p; la.v_sss = c->model.v_sss;
  la.v_sps = c->model.v_sps; la.v_pps = c->model.v_pps; la.v_ppp = c->model.v_ppp;
  la.vbuf = c->vbuf; la.tab = c->tab; la.kused = c->kused; la.vj = c->vj;
  la.counter = c->work_counter; la.stats = c->stats;
  la.omega = c->omega;
  // re-orthogonalisation threshold on the estimated |V_j^T V_{k+1}|: well
  // below the parity bar in FP64; in FP32 at the level the FP32 recursion
  // already carries
  la.eta = fp32 ? 1e-4 : 1e-12;
  // BF16 operands perturb every product by ~2^-8 relative: the estimate's
  // rounding term uses the BF16 epsilon, so the passes run at every step
  la.eps_unit = precision == TB_BF16 ? 0.0078125 : (fp32 ? (double)FLT_EPSILON : DBL_EPSILON);
  la.om_lds = la.ab_lds = la.vprev_lds = 0;
  la.scalar = c->seeds == TB_SEEDS_ORBITAL ? 1 : 0;
  return la;
}

static EigArgs eig_args(const tb_ctx* c, int n, int precision) {
  EigArgs ea;
  ea.u_fp32 = precision != TB_FP64 ? 1 : 0;      // U in the recursion's precision (k_rho reads it so)
  ea.atom0 = 0; ea.n_atoms = n; ea.r_max = c->r_max; ea.tab = c->tab; ea.kused = c->kused;
  ea.lam = c->lam; ea.wgt = c->wgt; ea.y1 = c->y1;
  ea.ref_v = c->ref_v; ea.ref_p = c->ref_p; ea.ref_n = c->ref_n; ea.ref_max = c->ref_max;
  ea.seg = c->seg; ea.seg_n = c->seg_n; ea.seg_max = c->seg_max;
  ea.counter = c->work_counter + 1; ea.scratch = c->eig_scratch; ea.evec = c->evec; ea.vsc = c->vsc; ea.tri = c->tri;
  ea.stats = c->stats;
  ea.scalar = c->seeds == TB_SEEDS_ORBITAL ? 1 : 0;
  return ea;
}

static int check_krylov_args(const tb_ctx* c, int r, int precision) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (c->stage < 1) return fail(TB_ESTATE, "tb_build_local_H must be called first");
  if (r < 1 || r > c->r_max) return fail(TB_ECAPACITY, "r=%d outside [1, %d]", r, c->r_max);
  if (precision != TB_FP64 && precision != TB_FP32 && precision != TB_BF16)
    return fail(TB_EINVAL, "unknown precision %d", precision);
  return TB_OK;
}

extern "C" int tb_krylov_rho(tb_ctx* c, int r, const int* r_per_atom, double kT, double mu, double n_electrons,
                             int precision, double* mu_out, double* rho_out) {
  const int bad = check_krylov_args(c, r, precision);
  if (bad) return bad;
  if (!rho_out) return fail(TB_EINVAL, "rho_out is null");
  if (!(isfinite(kT) && kT > 0)) return fail(TB_EINVAL, "kT must be positive and finite");
  const bool fixed = !isnan(mu);
  if (fixed && !isfinite(mu)) return fail(TB_EINVAL, "mu must be finite or NaN");
  const int n = (int)c->n_atoms;
  if (!fixed && !(isfinite(n_electrons) && n_electrons > 0 && n_electrons < 8.0 * n))
    return fail(TB_EMU, "n_electrons=%g outside (0, %d)", n_electrons, 8 * n);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  c->kT = kT;
  c->precision = precision;
  const bool fp32 = precision != TB_FP64;      // FP32 recursion (TB_FP32, TB_BF16)
  // K4: block Lanczos
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, c->work_counter, 16);
  LanczosArgs la = lanczos_args(c, n, r, r_per_atom, precision);
  const LzPlan plan = lanczos_plan(c, fp32, c->lz_nt[precision], c->lz_minw[precision], c->lz_per_cu[precision]);
  la.om_lds = plan.om_lds; la.ab_lds = plan.ab_lds; la.vprev_lds = plan.vprev_lds;
  // per-atom phases run over consecutive groups of `chunk` target atoms, one
  // launch per group (a single group by default); persistent kernels take a
  // freshly zeroed queue counter per launch
  const int chunk = c->atoms_per_launch > 0 && c->atoms_per_launch < n ? c->atoms_per_launch : n;
  int pk = prof_begin(c, 1);
  for (int a0 = 0; a0 < n; a0 += chunk) {
    const int a1 = n - a0 > chunk ? a0 + chunk : n;
    if (a0 > 0) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, c->work_counter, 1);
    la.atom0 = a0; la.n_atoms = a1;
    launch_lanczos(la, precision, plan.nt, plan.minw, c->lz_wide[precision],
                   plan.n_wg < a1 - a0 ? plan.n_wg : a1 - a0, plan.lds, st);
  }
  prof_end(c, pk);
  // K5: projected eigensolve
  EigArgs ea = eig_args(c, n, precision);
  pk = prof_begin(c, 2);
  for (int a0 = 0; a0 < n; a0 += chunk) {
    const int a1 = n - a0 > chunk ? a0 + chunk : n;
    if (a0 > 0) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, c->work_counter + 1, 1);
    ea.atom0 = a0; ea.n_atoms = a1;
    const int n_wg_eig = c->n_cu * c->eig_per_cu;
    launch_eig(ea, n_wg_eig < a1 - a0 ? n_wg_eig : a1 - a0, st);
  }
  prof_end(c, pk);
  // K6: chemical potential and spectral sums
  MuArgs ma;
  ma.n_pairs = (int64_t)n * 4 * c->r_max;
  ma.lam = c->lam; ma.wgt = c->wgt; ma.kT = kT; ma.n_e = n_electrons;
  ma.state = c->mu_state; ma.partial = c->partial;
  ma.eparts = c->eparts; ma.mu_out = mu_out;
  pk = prof_begin(c, 3);
  launch_mu(ma, mu, fixed, MU_ITERS, st);
  prof_end(c, pk);
  // K7: density-matrix blocks
  RhoArgs ra;
  ra.n_atoms = n; ra.r_max = c->r_max; ra.kused = c->kused; ra.hop_n = c->hop_n; ra.clu_j = c->clu_j;
  ra.nc_max = c->nc_max; ra.zmax = c->zmax; ra.lam = c->lam; ra.y1 = c->y1; ra.ref_v = c->ref_v; ra.ref_p = c->ref_p;
  ra.ref_n = c->ref_n; ra.ref_max = c->ref_max;
  ra.seg = c->seg; ra.seg_n = c->seg_n; ra.seg_max = c->seg_max; ra.evec = c->evec; ra.vsc = c->vsc; ra.vj = c->vj; ra.vj_fp32 = fp32 ? 1 : 0;
  ra.row_ptr = c->row_ptr; ra.mu_state = c->mu_state; ra.kT = kT; ra.rho = rho_out; ra.stats = c->stats;
  pk = prof_begin(c, 4);
  for (int a0 = 0; a0 < n; a0 += chunk) {
    ra.atom0 = a0; ra.n_atoms = n - a0 > chunk ? a0 + chunk : n;
    launch_rho(ra, st);
  }
  prof_end(c, pk);
  HIP_TRY(hipGetLastError());
  c->rho_last = rho_out;
  c->stage = 2;
  c->have_virial = 0;
  return TB_OK;
}

// Launch-shape tuner: times the Krylov kernel for every shape that fits
// (threads per workgroup x persistent workgroups per compute unit) and then
// k_band + k_eig for every k_eig occupancy, on this context's current spheres;
// each candidate runs twice and its faster run counts. The choice changes
// launch geometry, registers and LDS residency; the thread count also sets
// the order of the workgroup reductions, so results move at rounding level.
extern "C" int tb_autotune(tb_ctx* c, int r, const int* r_per_atom, int precision, int* shape_out) {
  const int bad = check_krylov_args(c, r, precision);
  if (bad) return bad;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const bool fp32 = precision != TB_FP64;
  const int n = (int)c->n_atoms;
  int64_t saved[ST_NSTATS];
  HIP_TRY(hipMemcpyAsync(saved, c->stats, sizeof saved, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto timed = [&](auto&& launch, float& best_ms) -> hipError_t {
    for (int rep = 0; rep < 2; ++rep) {
      hipEventRecord(e0, st);
      launch();
      hipEventRecord(e1, st);
      hipError_t e = hipEventSynchronize(e1);
      if (e != hipSuccess) return e;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) return e;
      if (ms < best_ms) best_ms = ms;
    }
    return hipGetLastError();
  };
  LanczosArgs la = lanczos_args(c, n, r, r_per_atom, precision);
  int best_nt = c->lz_nt[precision], best_mw = c->lz_minw[precision], best_pc = c->lz_per_cu[precision];
  int best_wide = c->lz_wide[precision];
  int tried = 0;
  float best = 3.0e38f;
  hipError_t err = hipSuccess;
  const int nts[2] = {256, 512}, mws[3] = {4, 3, 2};   // waves per SIMD (3: 256 threads only)
  // H.V item layouts: FP32 all four, FP64 the four-lanes-per-atom (0) and
  // atom-per-lane (3) items, BF16 the one-column items
  const int layouts[4] = {0, 1, 2, 3}, layouts64[2] = {0, 3};
  const int n_wide = precision == TB_FP32 ? 4 : (precision == TB_FP64 ? 2 : 1);
  for (int wi = 0; wi < n_wide && err == hipSuccess; ++wi)
  for (int m = 0; m < 3 && err == hipSuccess; ++m) {
    const int wd = precision == TB_FP64 ? layouts64[wi] : layouts[wi];
    for (int q = 0; q < 2 && err == hipSuccess; ++q) {
      if (mws[m] == 3 && nts[q] != 256) continue;
      for (int pc = 1; pc <= c->lz_per_cu_max && err == hipSuccess; ++pc) {
        // co-resident only: waves per SIMD within the register budget
        if (pc * nts[q] / 64 > 4 * mws[m]) continue;
        const LzPlan p = lanczos_plan(c, fp32, nts[q], mws[m], pc);
        if (!p.lds) continue;
        la.om_lds = p.om_lds; la.ab_lds = p.ab_lds; la.vprev_lds = p.vprev_lds;
        float t = 3.0e38f;
        err = timed([&] {
          hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, c->work_counter, 16);
          launch_lanczos(la, precision, p.nt, p.minw, wd, p.n_wg < n ? p.n_wg : n, p.lds, st);
        }, t);
        ++tried;
        if (t < best) { best = t; best_nt = p.nt; best_mw = p.minw; best_pc = pc; best_wide = wd; }
      }
    }
  }
  int best_e = c->eig_per_cu;
  if (err == hipSuccess) {
    c->lz_nt[precision] = best_nt;
    c->lz_minw[precision] = best_mw;
    c->lz_per_cu[precision] = best_pc;
    c->lz_wide[precision] = best_wide;
    // k_eig consumes the recursion of the last Krylov run (identical for every shape)
    EigArgs ea = eig_args(c, n, precision);
    const int cand[5] = {2, 3, 4, 6, 8};
    float beste = 3.0e38f;
    for (int q = 0; q < 5 && err == hipSuccess; ++q) {
      if (cand[q] > c->eig_per_cu_max) continue;
      const int nw = c->n_cu * cand[q];
      float t = 3.0e38f;
      err = timed([&] {
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, c->work_counter, 16);
        launch_eig(ea, nw < n ? nw : n, st);
      }, t);
      ++tried;
      if (t < beste) { beste = t; best_e = cand[q]; }
    }
    if (err == hipSuccess) c->eig_per_cu = best_e;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return fail(TB_EHIP, "autotune: %s", hipGetErrorString(err));
  HIP_TRY(hipMemcpyAsync(c->stats, saved, sizeof saved, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  c->stage = 1;                      // the tuning runs replaced the recursion outputs
  c->have_virial = 0;
  if (shape_out) {
    shape_out[0] = c->lz_nt[precision];
    shape_out[1] = c->lz_per_cu[precision];
    shape_out[2] = c->eig_per_cu;
    shape_out[3] = tried;
    shape_out[4] = c->lz_minw[precision];
    shape_out[5] = c->lz_wide[precision];
  }
  return TB_OK;
}

extern "C" int tb_rho_layout(tb_ctx* c, int64_t* nnz_pairs_host, int64_t* row_ptr, int* col_j) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (c->stage < 1) return fail(TB_ESTATE, "tb_build_local_H must be called first");
  if (!nnz_pairs_host) return fail(TB_EINVAL, "nnz_pairs_host is null");
  HIP_TRY(hipSetDevice(c->device));
  int64_t nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, c->row_ptr + c->n_atoms, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *nnz_pairs_host = nnz;
  c->nnz_pairs = nnz;
  if (row_ptr)
    HIP_TRY(hipMemcpyAsync(row_ptr, c->row_ptr, (c->n_atoms + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                           c->stream));
  if (col_j) HIP_TRY(hipMemcpyAsync(col_j, c->col_j, nnz * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  return TB_OK;
}

static ForceArgs force_args(const tb_ctx* c) {
  ForceArgs fa;
  fa.n_atoms = (int)c->n_atoms; fa.zmax = c->zmax; fa.M = c->model;
  fa.hop_n = c->hop_n; fa.hop_j = c->hop_j; fa.hop_rev = c->hop_rev; fa.hop_d = c->hop_d;
  fa.row_ptr = c->row_ptr; fa.rho = c->rho_last; fa.xrep = c->xrep; fa.forces = nullptr;
  fa.grad_scale = nullptr; fa.eparts = c->eparts; fa.kT = c->kT; fa.e_out = nullptr;
  fa.wpart = c->wpart; fa.virial = c->virial;
  return fa;
}

extern "C" int tb_energy_forces(tb_ctx* c, double* e_out, double* forces) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (c->stage < 2) return fail(TB_ESTATE, "tb_krylov_rho must be called first");
  if (!e_out) return fail(TB_EINVAL, "e_out is null");
  HIP_TRY(hipSetDevice(c->device));
  ForceArgs fa = force_args(c);
  fa.forces = forces; fa.e_out = e_out;
  const int pk = prof_begin(c, 5);
  launch_forces(fa, forces != nullptr, c->stream);
  prof_end(c, pk);
  HIP_TRY(hipGetLastError());
  c->have_virial = forces != nullptr;
  return TB_OK;
}

extern "C" int tb_energy_forces_static(tb_ctx* c, double* e_out, double* forces) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (c->stage < 2) return fail(TB_ESTATE, "tb_krylov_rho must be called first");
  if (!e_out) return fail(TB_EINVAL, "e_out is null");
  const size_t need = static_scratch_need(c->n_atoms);
  if (need > static_scratch_bytes())
    return fail(TB_ECAPACITY, "%lld atoms need %zu B of fixed workspace; it holds %zu B",
                (long long)c->n_atoms, need, static_scratch_bytes());
  HIP_TRY(hipSetDevice(c->device));
  ForceArgs fa = force_args(c);
  if (!static_scratch_args(c->device, fa))
    return fail(TB_ESTATE, "fixed workspace of device %d not looked up", c->device);
  fa.forces = forces; fa.e_out = e_out;
  const int pk = prof_begin(c, 5);
  launch_forces(fa, forces != nullptr, c->stream);
  prof_end(c, pk);
  HIP_TRY(hipGetLastError());
  c->have_virial = forces != nullptr;
  return TB_OK;
}

extern "C" int tb_energy_backward(tb_ctx* c, const double* grad_e, double* grad_pos) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (!grad_e || !grad_pos) return fail(TB_EINVAL, "grad_e and grad_pos must not be null");
  if (c->stage < 2) return fail(TB_ESTATE, "tb_krylov_rho must be called first");
  HIP_TRY(hipSetDevice(c->device));
  ForceArgs fa = force_args(c);
  fa.forces = grad_pos; fa.grad_scale = grad_e;
  const int pk = prof_begin(c, 5);
  launch_forces(fa, true, c->stream);
  prof_end(c, pk);
  HIP_TRY(hipGetLastError());
  c->have_virial = 1;
  return TB_OK;
}

extern "C" int tb_virial(tb_ctx* c, double* virial_out) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (!virial_out) return fail(TB_EINVAL, "virial_out is null");
  if (c->stage < 2 || !c->have_virial) return fail(TB_ESTATE, "tb_energy_forces must be called first");
  HIP_TRY(hipSetDevice(c->device));
  launch_virial_copy(c->virial, virial_out, c->stream);
  HIP_TRY(hipGetLastError());
  return TB_OK;
}

extern "C" int tb_get_stats(tb_ctx* c, int64_t* stats_host, int n_stats) {
  if (!c || !stats_host) return fail(TB_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device));
  int64_t s[ST_NSTATS];
  HIP_TRY(hipMemcpyAsync(s, c->stats, sizeof s, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  s[ST_MEMORY] = (int64_t)c->bytes;
  for (int q = 0; q < n_stats && q < ST_NSTATS; ++q) stats_host[q] = s[q];
  if (s[ST_FLAGS] & FL_GROUP_IMAGE)
    return fail(TB_ECUTOFF, "a group's spread plus r_cluster reaches half a box length (flags 0x%llx)",
                (unsigned long long)s[ST_FLAGS]);
  if (s[ST_FLAGS] & (FL_HOP_OVERFLOW | FL_CLUSTER_OVERFLOW | FL_COUPLING_OVERFLOW))
    return fail(TB_ECAPACITY, "device list overflow (flags 0x%llx)", (unsigned long long)s[ST_FLAGS]);
  if (s[ST_FLAGS]) return fail(TB_EDEVICE, "device error flags 0x%llx", (unsigned long long)s[ST_FLAGS]);
  return TB_OK;
}

extern "C" int tb_set_seeds(tb_ctx* c, int seeds) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (seeds != TB_SEEDS_BLOCK && seeds != TB_SEEDS_ORBITAL) return fail(TB_EINVAL, "unknown seeds %d", seeds);
  c->seeds = seeds;
  return TB_OK;
}

extern "C" int tb_set_groups(tb_ctx* c, int m) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (m < 1 || m > GROUP_MAX) return fail(TB_EINVAL, "group size %d outside [1, %d]", m, GROUP_MAX);
  if ((int64_t)m * c->nc_max > UNION_LDS_MAX)
    return fail(TB_ECAPACITY, "group size %d x sphere capacity %d exceeds %d", m, c->nc_max, UNION_LDS_MAX);
  c->group_m = m;
  c->stage = 0;                               // the spheres must be rebuilt
  return TB_OK;
}

extern "C" int tb_set_shape(tb_ctx* c, int precision, int threads, int waves_per_simd, int wg_per_cu, int wide) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (precision != TB_FP64 && precision != TB_FP32 && precision != TB_BF16)
    return fail(TB_EINVAL, "unknown precision %d", precision);
  if (threads != 256 && threads != 512) return fail(TB_EINVAL, "threads=%d is not 256 or 512", threads);
  if (waves_per_simd != 2 && waves_per_simd != 3 && waves_per_simd != 4)
    return fail(TB_EINVAL, "waves_per_simd=%d is not 2, 3 or 4", waves_per_simd);
  if (waves_per_simd == 3 && threads != 256) return fail(TB_EINVAL, "waves_per_simd=3 needs 256 threads");
  if (wg_per_cu < 1 || wg_per_cu > c->lz_per_cu_max)
    return fail(TB_EINVAL, "wg_per_cu=%d outside [1, %d]", wg_per_cu, c->lz_per_cu_max);
  if (wide < 0 || wide > 3) return fail(TB_EINVAL, "H.V layout %d is not 0, 1, 2 or 3", wide);
  if ((wide == 1 || wide == 2) && precision != TB_FP32)
    return fail(TB_EINVAL, "the wide and MFMA H.V layouts are for TB_FP32 only");
  if (wide == 3 && precision == TB_BF16) return fail(TB_EINVAL, "the BF16 form has the one-column H.V layout only");
  if (wg_per_cu * threads / 64 > 4 * waves_per_simd)
    return fail(TB_EINVAL, "%d workgroups of %d threads exceed %d waves per SIMD", wg_per_cu, threads,
                waves_per_simd);
  if (!lanczos_plan(c, precision != TB_FP64, threads, waves_per_simd, wg_per_cu).lds)
    return fail(TB_ECAPACITY, "the sphere capacity does not fit %d workgroups per compute unit", wg_per_cu);
  c->lz_nt[precision] = threads;
  c->lz_minw[precision] = waves_per_simd;
  c->lz_per_cu[precision] = wg_per_cu;
  c->lz_wide[precision] = wide;
  return TB_OK;
}

extern "C" int tb_set_launch(tb_ctx* c, int atoms_per_launch) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  if (atoms_per_launch < 0) return fail(TB_EINVAL, "atoms_per_launch=%d < 0", atoms_per_launch);
  c->atoms_per_launch = atoms_per_launch;
  return TB_OK;
}

extern "C" int tb_profile_enable(tb_ctx* c, int enable) {
  if (!c) return fail(TB_EINVAL, "ctx is null");
  HIP_TRY(hipSetDevice(c->device));
  if (enable && !c->ev_pool) {
    c->ev_pool = new hipEvent_t[2 * PROF_MAX];
    c->ev_phase = new int[PROF_MAX];
    for (int k = 0; k < 2 * PROF_MAX; ++k) HIP_TRY(hipEventCreate(&c->ev_pool[k]));
  }
  c->prof = enable ? 1 : 0;
  return TB_OK;
}

extern "C" int tb_profile_read(tb_ctx* c, double* ms_host, int64_t* count_host, int n) {
  if (!c || !ms_host || !count_host || n < N_PHASES) return fail(TB_EINVAL, "null argument or n < 6");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
    ms_host[c->ev_phase[k]] += ms;
    count_host[c->ev_phase[k]] += 1;
  }
  if (n > N_PHASES) count_host[N_PHASES] += c->ev_dropped;
  c->ev_used = 0;
  c->ev_dropped = 0;
  return TB_OK;
}
