// Context life cycle, mesh set-up (geometry, colouring, node-block sparsity
// pattern), material table and boundary data.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "common.hpp"

using namespace hfsi;

namespace {

constexpr int NBR_MAX = 512;  // distinct neighbours of one node (incl. itself)

// Reference gradients of the P1 hat functions, volume and longest edge of
// every tetrahedron: with D = [X1-X0, X2-X0, X3-X0], grad N_a (a = 1..3) is
// row a-1 of D^{-1} and grad N_0 is minus their sum.
__global__ void k_geometry(int m, const int* __restrict__ T, const double* __restrict__ X,
                           double* __restrict__ G, double* __restrict__ V, double* __restrict__ H,
                           int* __restrict__ bad) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double x[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int nd = T[a * m + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) x[a][i] = X[3 * nd + i];
  }
  double D[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) D[i][j] = x[j + 1][i] - x[0][i];
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  if (!(det > 0.0)) atomicOr(bad, 1);
  const double id = 1.0 / det;
  // inverse = adjugate / det (row r of the inverse = gradient of N_{r+1})
  double Di[3][3];
  Di[0][0] = c00 * id;
  Di[1][0] = c01 * id;
  Di[2][0] = c02 * id;
  Di[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
  Di[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
  Di[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
  Di[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
  Di[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
  Di[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
#pragma unroll
  for (int J = 0; J < 3; ++J) {
    G[(0 * 3 + J) * m + e] = -(Di[0][J] + Di[1][J] + Di[2][J]);
    G[(1 * 3 + J) * m + e] = Di[0][J];
    G[(2 * 3 + J) * m + e] = Di[1][J];
    G[(3 * 3 + J) * m + e] = Di[2][J];
  }
  V[e] = det / 6.0;
  double hm = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b) {
      double dx = x[a][0] - x[b][0], dy = x[a][1] - x[b][1], dz = x[a][2] - x[b][2];
      hm = fmax(hm, sqrt(dx * dx + dy * dy + dz * dz));
    }
  H[e] = hm;
}

__global__ void k_node_deg(int m, const int* __restrict__ T, int* __restrict__ deg) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  for (int a = 0; a < 4; ++a) atomicAdd(&deg[T[a * m + e]], 1);
}

__global__ void k_node_fill(int m, const int* __restrict__ T, const int* __restrict__ ptr,
                            int* __restrict__ cursor, int* __restrict__ n2t) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  for (int a = 0; a < 4; ++a) {
    int nd = T[a * m + e];
    int pos = ptr[nd] + atomicAdd(&cursor[nd], 1);
    n2t[pos] = e;
  }
}

// Sorted distinct nodes sharing a tetrahedron with node i (sort-reduce of the
// candidate list gathered from the incident elements).  fill == false: count.
__global__ void k_node_nbrs(int n, int m, const int* __restrict__ T, const int* __restrict__ n2t_ptr,
                            const int* __restrict__ n2t, int* __restrict__ cnt, const int* __restrict__ nptr,
                            int* __restrict__ ncol, int* __restrict__ overflow, bool fill) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int list[NBR_MAX];
  int k = 0;
  for (int q = n2t_ptr[i]; q < n2t_ptr[i + 1]; ++q) {
    int e = n2t[q];
    for (int a = 0; a < 4; ++a) {
      int nd = T[a * m + e];
      // insertion into the sorted list, skipping duplicates
      int pos = k;
      bool dup = false;
      for (int s = 0; s < k; ++s) {
        if (list[s] == nd) { dup = true; break; }
        if (list[s] > nd) { pos = s; break; }
      }
      if (dup) continue;
      if (k == NBR_MAX) { atomicOr(overflow, 1); return; }
      for (int s = k; s > pos; --s) list[s] = list[s - 1];
      list[pos] = nd;
      ++k;
    }
  }
  if (!fill) {
    cnt[i] = k;
  } else {
    int base = nptr[i];
    for (int s = 0; s < k; ++s) ncol[base + s] = list[s];
  }
}

__device__ __forceinline__ int find_sorted(const int* __restrict__ a, int lo, int hi, int key) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_slots(int m, const int* __restrict__ T, const int* __restrict__ nptr, const int* __restrict__ ncol,
                        int* __restrict__ slot) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int nd[4];
  for (int a = 0; a < 4; ++a) nd[a] = T[a * m + e];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      slot[(a * 4 + b) * m + e] = find_sorted(ncol, nptr[nd[a]], nptr[nd[a] + 1], nd[b]);
}

__global__ void k_diag_blk(int n, const int* __restrict__ nptr, const int* __restrict__ ncol, int* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = find_sorted(ncol, nptr[i], nptr[i + 1], i);
}

__global__ void k_block_rows(int n, const int* __restrict__ nptr, int* __restrict__ brow) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = nptr[i]; q < nptr[i + 1]; ++q) brow[q] = i;
}

// Consistent P1 mass on the node pattern, one colour at a time:
// M_ab = V (1 + delta_ab) / 20.
__global__ void k_mass_colour(int e0, int e1, int m, const int* __restrict__ slot, const double* __restrict__ V,
                              double* __restrict__ Mval) {
  int e = e0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  const double v20 = V[e] / 20.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Mval[slot[(a * 4 + b) * m + e]] += (a == b ? 2.0 : 1.0) * v20;
}

// Schur diagonal of eq. lpreschur: s_i = sum_T (1/theta_T + 1/kappa_T) V_T / 10
// (the diagonal of the consistent P1 pressure mass is V/10 per node).
__global__ void k_schur_colour(int e0, int e1, int m, const int* __restrict__ T, const int* __restrict__ mat,
                               const double* __restrict__ mtab, const double* __restrict__ V,
                               double* __restrict__ s) {
  int e = e0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  const double* mt = mtab + 8 * mat[e];
  const double w = (1.0 / mt[7] + 1.0 / mt[3]) * V[e] / 10.0;
  for (int a = 0; a < 4; ++a) s[T[a * m + e]] += w;
}

// Nodal load of the dead traction: f_a = sum_{tri contains a} t_tri A_tri / 3,
// gathered per node over its incident loaded triangles.
__global__ void k_loads(int n, const int* __restrict__ n2tri_ptr, const int* __restrict__ n2tri,
                        const int* __restrict__ tris, const double* __restrict__ trac,
                        const double* __restrict__ X, double* __restrict__ f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int q = n2tri_ptr[i]; q < n2tri_ptr[i + 1]; ++q) {
    int t = n2tri[q];
    const double* p0 = X + 3 * tris[3 * t + 0];
    const double* p1 = X + 3 * tris[3 * t + 1];
    const double* p2 = X + 3 * tris[3 * t + 2];
    double ux = p1[0] - p0[0], uy = p1[1] - p0[1], uz = p1[2] - p0[2];
    double vx = p2[0] - p0[0], vy = p2[1] - p0[1], vz = p2[2] - p0[2];
    double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    double area3 = 0.5 * sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
    fx += trac[3 * t + 0] * area3;
    fy += trac[3 * t + 1] * area3;
    fz += trac[3 * t + 2] * area3;
  }
  f[3 * i + 0] = fx;
  f[3 * i + 1] = fy;
  f[3 * i + 2] = fz;
}

// Greedy element colouring: no two elements of one colour share a node.
// Each node keeps bit masks of the colours already touching it, 64 colours
// per word; a word is added when every colour of the earlier ones is taken
// at some element (meshes with a node in many elements, such as the axis
// of a lumen mesh), up to 1024 colours.
void colour_elements(int n, int m, const int32_t* tets, std::vector<int>& perm, std::vector<int>& cptr) {
  constexpr size_t kMaxWords = 16;
  std::vector<std::vector<uint64_t>> used(1, std::vector<uint64_t>(n, 0));
  std::vector<int> col(m);
  int ncol = 0;
  for (int e = 0; e < m; ++e) {
    int c = -1;
    for (size_t w = 0; c < 0; ++w) {
      if (w == used.size()) {
        if (w >= kMaxWords) fail(HFSI_E_CAPACITY, "element colouring needs more than 1024 colours");
        used.emplace_back(n, 0);
      }
      uint64_t u = 0;
      for (int a = 0; a < 4; ++a) u |= used[w][tets[4 * e + a]];
      if (~u != 0) {
        const int b = __builtin_ctzll(~u);
        c = 64 * (int)w + b;
        for (int a = 0; a < 4; ++a) used[w][tets[4 * e + a]] |= (1ull << b);
      }
    }
    col[e] = c;
    ncol = std::max(ncol, c + 1);
  }
  cptr.assign(ncol + 1, 0);
  for (int e = 0; e < m; ++e) cptr[col[e] + 1]++;
  for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
  perm.assign(m, 0);
  std::vector<int> cur(cptr.begin(), cptr.end() - 1);
  for (int e = 0; e < m; ++e) perm[cur[col[e]]++] = e;
}

}  // namespace

// ================================================================== ABI

extern "C" int32_t hfsi_abi_version(void) { return 11; }

namespace {
std::atomic<int> g_live_contexts{0};  // the device block cache is trimmed when none is left

// events and pinned host memory of a context (safe on partly created ones)
void release_events(hfsi_ctx* c) {
  for (hipEvent_t* e : {&c->ev0, &c->ev1, &c->kev[0], &c->kev[1], &c->aev[0], &c->aev[1]})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
    c->aux = nullptr;
  }
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
}
}  // namespace

extern "C" hfsi_status hfsi_create(hfsi_ctx** out, int device, void* stream) {
  if (!out) return HFSI_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HFSI_E_ARG;
  hfsi_ctx* c = new hfsi_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  const bool ok = hipSetDevice(device) == hipSuccess && hipEventCreate(&c->ev0) == hipSuccess &&
                  hipEventCreate(&c->ev1) == hipSuccess &&
                  hipEventCreateWithFlags(&c->kev[0], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->kev[1], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->aev[0], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->aev[1], hipEventDisableTiming) == hipSuccess &&
                  hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess &&
                  hipHostMalloc((void**)&c->pinned, 64 * sizeof(double)) == hipSuccess;
  if (!ok) {
    release_events(c);
    delete c;
    return HFSI_E_HIP;
  }
  try {
    hfsi::noalloc_scratch_init(device);
  } catch (const hfsi::Error&) {
    release_events(c);
    delete c;
    return HFSI_E_HIP;
  }
  *out = c;
  ++g_live_contexts;
  return HFSI_OK;
}

extern "C" hfsi_status hfsi_destroy(hfsi_ctx* c) {
  if (!c) return HFSI_E_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->aux) (void)hipStreamSynchronize(c->aux);
  // the streams are idle: the context's device blocks become free for any stream
  hfsi::tls_stream = c->stream;
  hfsi::tls_idle = true;
  release_events(c);
  hfsi::mlp_free(c);
  hfsi::vanka_free(c);
  hfsi::fluid_free(c);
  delete c;
  hfsi::tls_idle = false;
  if (--g_live_contexts == 0) hfsi::dev_cache_trim();
  return HFSI_OK;
}

extern "C" const char* hfsi_last_error(const hfsi_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" hfsi_status hfsi_set_mesh(hfsi_ctx* c, int64_t n_nodes, const double* X, int64_t n_tets,
                                     const int32_t* tets, const int32_t* mat_id, const int32_t* lattice,
                                     const double* fibres) {
  HFSI_ABI_BEGIN(c)
  if (n_nodes <= 0 || n_tets <= 0 || !X || !tets || !mat_id) fail(HFSI_E_ARG, "set_mesh: empty mesh or null array");
  if (n_nodes > (1 << 29) || n_tets > (1 << 27)) fail(HFSI_E_ARG, "set_mesh: mesh too large for int32 indexing");
  const int n = (int)n_nodes, m = (int)n_tets;
  int max_mat = 0;
  for (int e = 0; e < m; ++e) {
    for (int a = 0; a < 4; ++a)
      if (tets[4 * e + a] < 0 || tets[4 * e + a] >= n) fail(HFSI_E_ARG, "set_mesh: node index out of range");
    if (mat_id[e] < 0) fail(HFSI_E_ARG, "set_mesh: negative material id");
    max_mat = std::max(max_mat, (int)mat_id[e]);
  }
  hipStream_t s = c->stream;
  c->n = n;
  c->m = m;
  c->stage = 0;
  c->H.ready = false;
  hfsi::vanka_invalidate(c);
  c->H.reusable = false;
  c->nm_rho = 0.0;  // a new mesh starts quasi-static, as a structure
  c->cm = 0.0;
  c->rs.release();
  hfsi::fluid_free(c);
  colour_elements(n, m, tets, c->perm, c->colour_ptr);

  // element arrays in colour order, structure of arrays
  std::vector<int> T(4 * (size_t)m), mt(m);
  std::vector<double> fb;
  c->has_fib = fibres != nullptr;
  if (c->has_fib) fb.resize(6 * (size_t)m);
  for (int k = 0; k < m; ++k) {
    int e = c->perm[k];
    for (int a = 0; a < 4; ++a) T[(size_t)a * m + k] = tets[4 * e + a];
    mt[k] = mat_id[e];
    if (c->has_fib)
      for (int q = 0; q < 6; ++q) fb[(size_t)q * m + k] = fibres[6 * e + q];
  }
  c->X.upload(X, 3 * (size_t)n, s);
  c->tets.upload(T.data(), T.size(), s);
  c->mat.upload(mt.data(), mt.size(), s);
  if (c->has_fib) c->fib.upload(fb.data(), fb.size(), s); else c->fib.release();
  c->has_lattice = lattice != nullptr;
  if (c->has_lattice) c->lattice.upload(lattice, 3 * (size_t)n, s); else c->lattice.release();

  // geometry
  c->G.ensure(12 * (size_t)m);
  c->V.ensure(m);
  c->h.ensure(m);
  DevBuf<int> flag;
  flag.zero(4, s);
  k_geometry<<<div_up(m, 256), 256, 0, s>>>(m, c->tets.p, c->X.p, c->G.p, c->V.p, c->h.p, flag.p);
  HIP_LAUNCH_CHECK();

  // node -> element lists
  DevBuf<int> deg, n2t_ptr, cursor, n2t, cnt;
  deg.zero(n + 1, s);
  k_node_deg<<<div_up(m, 256), 256, 0, s>>>(m, c->tets.p, deg.p);
  HIP_LAUNCH_CHECK();
  n2t_ptr.ensure(n + 1);
  int64_t tot = exclusive_scan(deg.p, n2t_ptr.p, n + 1, s);
  if (tot != 4 * (int64_t)m) fail(HFSI_E_HIP, "set_mesh: incidence count mismatch");
  cursor.zero(n, s);
  n2t.ensure(4 * (size_t)m);
  k_node_fill<<<div_up(m, 256), 256, 0, s>>>(m, c->tets.p, n2t_ptr.p, cursor.p, n2t.p);
  HIP_LAUNCH_CHECK();

  // node-block pattern by sort-reduce of each node's candidate list
  cnt.zero(n + 1, s);
  k_node_nbrs<<<div_up(n, 128), 128, 0, s>>>(n, m, c->tets.p, n2t_ptr.p, n2t.p, cnt.p, nullptr, nullptr,
                                            flag.p + 1, false);
  HIP_LAUNCH_CHECK();
  c->nptr.ensure(n + 1);
  int64_t nb = exclusive_scan(cnt.p, c->nptr.p, n + 1, s);
  if (16 * nb > INT32_MAX) fail(HFSI_E_ARG, "set_mesh: tangent exceeds int32 indexing");
  c->nb = (int)nb;
  c->ncol.ensure(nb);
  k_node_nbrs<<<div_up(n, 128), 128, 0, s>>>(n, m, c->tets.p, n2t_ptr.p, n2t.p, nullptr, c->nptr.p, c->ncol.p,
                                            flag.p + 1, true);
  HIP_LAUNCH_CHECK();
  c->slot.ensure(16 * (size_t)m);
  k_slots<<<div_up(m, 256), 256, 0, s>>>(m, c->tets.p, c->nptr.p, c->ncol.p, c->slot.p);
  HIP_LAUNCH_CHECK();
  c->diag_blk.ensure(n);
  k_diag_blk<<<div_up(n, 256), 256, 0, s>>>(n, c->nptr.p, c->ncol.p, c->diag_blk.p);
  HIP_LAUNCH_CHECK();
  c->Kval.ensure(16 * (size_t)nb);
  c->brow.ensure(nb);
  k_block_rows<<<div_up(n, 256), 256, 0, s>>>(n, c->nptr.p, c->brow.p);
  HIP_LAUNCH_CHECK();

  // consistent mass on the pattern
  c->Mval.zero(nb, s);
  for (size_t q = 0; q + 1 < c->colour_ptr.size(); ++q) {
    int e0 = c->colour_ptr[q], e1 = c->colour_ptr[q + 1];
    k_mass_colour<<<div_up(e1 - e0, 256), 256, 0, s>>>(e0, e1, m, c->slot.p, c->V.p, c->Mval.p);
    HIP_LAUNCH_CHECK();
  }
  auto f = flag.download(4, s);
  if (f[0]) fail(HFSI_E_ARG, "set_mesh: an element has non-positive volume (check orientation)");
  if (f[1]) fail(HFSI_E_CAPACITY, "set_mesh: a node has more than 511 neighbours");
  c->stage = 1;
  c->judge.valid = false;
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_set_materials(hfsi_ctx* c, int32_t n_mat, const hfsi_material* mats) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 1, "set_materials");
  if (n_mat <= 0 || !mats) fail(HFSI_E_ARG, "set_materials: empty table");
  auto mt = c->mat.download(c->m, c->stream);
  for (int v : mt)
    if (v >= n_mat) fail(HFSI_E_ARG, "set_materials: a material id exceeds the table");
  c->mtab_h.assign(8 * (size_t)n_mat, 0.0);
  for (int k = 0; k < n_mat; ++k) {
    const hfsi_material& q = mats[k];
    if (q.struct_size != sizeof(hfsi_material)) fail(HFSI_E_ARG, "set_materials: struct_size mismatch");
    if (q.model != 0 && q.model != 1) fail(HFSI_E_ARG, "set_materials: unknown model");
    if (!(q.c10 > 0) || !(q.kappa > 0)) fail(HFSI_E_ARG, "set_materials: c10 and kappa must be positive");
    double mu = q.model == 1 ? 2.0 * (q.c10 + (q.k2 > 0 ? q.k1 / (2.0 * q.k2) : 0.0)) : 2.0 * (q.c10 + q.c01);
    double* r = &c->mtab_h[8 * k];
    r[0] = q.model; r[1] = q.c10; r[2] = q.model == 0 ? q.c01 : 0.0; r[3] = q.kappa;
    // Schur parameter of eq. lpreschur: theta = O(c10), adjusted on a coarse
    // mesh and then kept (the fewest Krylov iterations on the 16^3 cube at
    // mu^l / 5); a positive theta in the record overrides it
    r[4] = q.k1; r[5] = q.k2; r[6] = mu; r[7] = q.theta > 0 ? q.theta : 0.2 * mu;
  }
  for (int k = 0; k < n_mat; ++k)
    if (c->mtab_h[8 * k] == 1 && !c->has_fib) fail(HFSI_E_ARG, "set_materials: artery model needs fibre directions");
  c->n_mat = n_mat;
  c->mtab.upload(c->mtab_h.data(), c->mtab_h.size(), c->stream);
  c->schur.zero(c->n, c->stream);
  for (size_t q = 0; q + 1 < c->colour_ptr.size(); ++q) {
    int e0 = c->colour_ptr[q], e1 = c->colour_ptr[q + 1];
    k_schur_colour<<<div_up(e1 - e0, 256), 256, 0, c->stream>>>(e0, e1, c->m, c->tets.p, c->mat.p, c->mtab.p,
                                                                 c->V.p, c->schur.p);
    HIP_LAUNCH_CHECK();
  }
  HIP_CHECK(hipStreamSynchronize(c->stream));
  c->stage = 2;
  c->judge.valid = false;
  c->keep_valid = false;  // a kept preconditioner belongs to the old material table
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_set_bc(hfsi_ctx* c, const uint8_t* dir_mask, int64_t n_tris, const int32_t* tris,
                                   const double* traction) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 2, "set_bc");
  if (!dir_mask || n_tris < 0 || (n_tris > 0 && (!tris || !traction))) fail(HFSI_E_ARG, "set_bc: bad arguments");
  const int n = c->n;
  std::vector<uint8_t> dm(dir_mask, dir_mask + 4 * (size_t)n);
  for (auto& v : dm) v = v ? 1 : 0;
  c->dir.upload(dm.data(), dm.size(), c->stream);
  // node -> loaded triangle lists (index bookkeeping on the host)
  std::vector<int> ptr(n + 1, 0), lst(3 * (size_t)n_tris);
  for (int64_t t = 0; t < n_tris; ++t)
    for (int a = 0; a < 3; ++a) {
      int nd = tris[3 * t + a];
      if (nd < 0 || nd >= n) fail(HFSI_E_ARG, "set_bc: triangle node out of range");
      ptr[nd + 1]++;
    }
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int> cur(ptr.begin(), ptr.end() - 1);
  for (int64_t t = 0; t < n_tris; ++t)
    for (int a = 0; a < 3; ++a) lst[cur[tris[3 * t + a]]++] = (int)t;
  DevBuf<int> dptr, dlst, dtris;
  DevBuf<double> dtr;
  dptr.upload(ptr.data(), ptr.size(), c->stream);
  dlst.upload(lst.data(), lst.size(), c->stream);
  dtris.upload(tris, 3 * (size_t)n_tris, c->stream);
  dtr.upload(traction, 3 * (size_t)n_tris, c->stream);
  c->fext.ensure(3 * (size_t)n);
  k_loads<<<div_up(n, 256), 256, 0, c->stream>>>(n, dptr.p, dlst.p, dtris.p, dtr.p, c->X.p, c->fext.p);
  HIP_LAUNCH_CHECK();
  build_a_pattern(c);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  c->stage = 3;
  c->judge.valid = false;
  c->H.ready = false;
  hfsi::vanka_invalidate(c);
  c->H.reusable = false;
  HFSI_ABI_END(c)
}
