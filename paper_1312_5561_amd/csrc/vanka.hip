// Coupled displacement-pressure AMG with the multiplicative Vanka smoother
// (section "AMG methods for the mixed problems", subsection "The
// multiplicative Vanka smoother", eq. locsys and eq. vankasmooth): the V-cycle
// acts on the whole linearised saddle-point system K = [A B1^T; B2 -C]
// (eq. globsys) and replaces the block preconditioner P_L when the AMG
// parameters ask for it (coupled = 1).
//
// Transfer: P = diag(P_u, P_p), P_u from the displacement hierarchy on A,
// P_p from a hierarchy built by the same strength / PMIS / interpolation on
// the pressure block C (one unknown per row); the shorter of the two
// continues with the identity.  Coarse blocks are Galerkin products on the
// structural product patterns; the coarsest coupled system is inverted by
// Gauss-Jordan with partial pivoting.
//
// Smoother: one patch per pressure unknown i = p_i plus the displacement
// unknowns of B2's row i.  Each patch's local matrix is factored once per
// set-up (LU with partial pivoting, one wavefront per patch) and its explicit
// inverse kept (column-major), so a local solve is one dense product with no
// sequential chain.  The patches are coloured first-fit in increasing index
// on the conflict graph pat(B2 A B1^T) + pat(C) (two patches conflict when K
// couples an unknown of one with an unknown of the other); a sweep runs the
// colours in order: per colour one launch forms the local residuals of all
// its patches (row-parallel over the whole chip) and one solves and updates
// (a 256-thread block per patch).  Patches of a colour share no unknown and
// no coupling, so this is the one-by-one Gauss-Seidel sweep in (colour,
// index) order.
//
// Additive variant (coupled = 2; the paper points to an additive form of the
// Vanka smoother without fixing its weights): every patch solves with the
// residual of the same iterate and each unknown takes omega times the mean
// of the corrections of the patches holding it.  A sweep is three launches
// whatever the colouring: the residual, all local solves (corrections kept
// per patch entry), and a per-unknown gather that adds its entries in patch
// order.  No colours are needed, so the set-up skips the conflict pattern.
//
// Every level stores its unknowns as [u (nu); p (np)].  fp64 throughout.
#include <algorithm>

#include "common.hpp"

namespace hfsi {

// amg.hip
int sparse_product(hfsi_ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& Cm, int* deferred);
void build_levels(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info);

namespace {

constexpr int kMaxPatch = 2048;     // unknowns of one patch (local system size)
constexpr int kMaxCoarsest = 4096;  // coupled coarsest system

struct VkLevel {
  int nu = 0, np = 0;
  const Csr<double>* Kuu = nullptr;  // operator of the displacement hierarchy
  const Csr<double>* C = nullptr;    // operator of the pressure hierarchy (C = -Kpp)
  Csr<double> Kup, Kpu;              // B1^T and B2 of this level
  const Csr<double>* Pu = nullptr;   // transfers to the next level (nullptr: identity)
  const Csr<double>* Ru = nullptr;
  const Csr<double>* Pp = nullptr;
  const Csr<double>* Rp = nullptr;
  int mmax = 0;                      // largest patch
  int lanes = 8;                     // lanes per row of the local residuals
  DevBuf<int> crow;                  // rows of the patches in sweep order
  DevBuf<int> roff;                  // [np + 1] first entry of each patch in crow
  std::vector<int> hroff;            // host copy
  DevBuf<double> rr;                 // local residuals of one colour
  DevBuf<int64_t> luoff;             // [np] first double of each patch's inverse
  DevBuf<double> inv;                // local inverses, column-major (fp64 hierarchy)
  DevBuf<float> inv32;               // the same rounded to fp32 (precision = 1; inv then released)
  std::vector<int> cptr;             // colour ranges of clist
  // the local solves' blocks: one per 64-row chunk of each patch, in sweep
  // order (q * 32 + chunk), and the first block of each colour
  DevBuf<int> work;
  std::vector<int> hwptr;
  DevBuf<int> clist;                 // patches in sweep order
  DevBuf<int> colour;                // [np] colour of each patch (export)
  DevBuf<double> x, b, r;            // [nu + np]
  // additive variant: the local corrections of all patch entries sorted by
  // unknown (each unknown's range [dptr[j], dptr[j+1]) in patch order), and
  // the slot in dd of every entry of crow
  DevBuf<double> dd;
  DevBuf<int> dptr, dpos;
};

struct Coupled {
  Hierarchy Hu, Hp;
  std::vector<VkLevel> L;
  // the V-cycle from L[0].b to L[0].x as one graph (thousands of small
  // launches: two per colour and sweep)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~Coupled() { drop_graph(); }
  int nc = 0;
  DevBuf<double> cinv;  // inverse of the coarsest coupled system, row-major
  double omega = 0.78;
  int steps = 6;
  bool additive = false;
  bool ready = false;
};

Coupled& state(hfsi_ctx* c) {
  if (!c->vanka_impl) c->vanka_impl = new Coupled();
  return *reinterpret_cast<Coupled*>(c->vanka_impl);
}

// ------------------------------------------------------------------ kernels

// level-0 blocks from the node-block tangent: Kup (3n x n), Kpu (n x 3n) and
// C = -Kpp (n x n), every stored block kept
__global__ void k_vk_ptr0(int n, const int* __restrict__ nptr, int* __restrict__ up_ptr, int* __restrict__ pu_ptr,
                          int* __restrict__ c_ptr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int b0 = nptr[i];
  if (i == n) {
    up_ptr[3 * n] = 3 * b0;
    pu_ptr[n] = 3 * b0;
    c_ptr[n] = b0;
    return;
  }
  const int deg = nptr[i + 1] - b0;
  for (int c = 0; c < 3; ++c) up_ptr[3 * i + c] = 3 * b0 + c * deg;
  pu_ptr[i] = 3 * b0;
  c_ptr[i] = b0;
}

__global__ void k_vk_blocks0(int nb, const int* __restrict__ brow, const int* __restrict__ nptr,
                             const int* __restrict__ ncol, const double* __restrict__ Kval, int* __restrict__ up_col,
                             double* __restrict__ up_val, int* __restrict__ pu_col, double* __restrict__ pu_val,
                             int* __restrict__ c_col, double* __restrict__ c_val) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb) return;
  const int i = brow[e], j = ncol[e];
  const int b0 = nptr[i], deg = nptr[i + 1] - b0, o = e - b0;
  const double* k = Kval + 16 * (size_t)e;
  for (int c = 0; c < 3; ++c) {
    const int q = 3 * b0 + c * deg + o;
    up_col[q] = j;
    up_val[q] = k[4 * c + 3];
    pu_col[3 * e + c] = 3 * j + c;
    pu_val[3 * e + c] = k[12 + c];
  }
  c_col[e] = j;
  c_val[e] = -k[15];
}

__global__ void k_vk_comp(int n, int three, int* __restrict__ comp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) comp[i] = three ? i % 3 : 0;
}

// local matrix of patch i (one 64-lane block per patch): rows and columns
// are the displacement unknowns U = B2 row i (sorted), then p_i
__global__ void __launch_bounds__(64) k_vk_build(int nu, const int* __restrict__ uu_ptr, const int* __restrict__ uu_col,
                                                 const double* __restrict__ uu_val, const int* __restrict__ up_ptr,
                                                 const int* __restrict__ up_col, const double* __restrict__ up_val,
                                                 const int* __restrict__ pu_ptr, const int* __restrict__ pu_col,
                                                 const double* __restrict__ pu_val, const int* __restrict__ c_ptr,
                                                 const int* __restrict__ c_col, const double* __restrict__ c_val,
                                                 const int64_t* __restrict__ luoff, double* __restrict__ lu) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const int p0 = pu_ptr[i], mu = pu_ptr[i + 1] - p0, m = mu + 1;
  double* M = lu + luoff[i];
  for (int t = lane; t < m * m; t += 64) M[t] = 0.0;
  __syncthreads();
  const int* U = pu_col + p0;
  for (int a = lane; a < m; a += 64) {
    if (a < mu) {
      const int j = U[a];
      for (int e = uu_ptr[j]; e < uu_ptr[j + 1]; ++e) {
        const int q = uu_col[e];
        int lo = 0, hi = mu;  // first position with U[pos] >= q
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (U[mid] < q) lo = mid + 1;
          else hi = mid;
        }
        if (lo < mu && U[lo] == q) M[(size_t)lo * m + a] = uu_val[e];
      }
      for (int e = up_ptr[j]; e < up_ptr[j + 1]; ++e)
        if (up_col[e] == i) M[(size_t)mu * m + a] = up_val[e];
    } else {
      for (int t = 0; t < mu; ++t) M[(size_t)t * m + mu] = pu_val[p0 + t];
      for (int e = c_ptr[i]; e < c_ptr[i + 1]; ++e)
        if (c_col[e] == i) M[(size_t)mu * m + mu] = -c_val[e];
    }
  }
}

// LU with partial pivoting of every patch's local matrix, in place
// (column-major; unit lower factor below the diagonal), and the row
// permutation: row k of the factored matrix is row perm[k] of the original
__global__ void __launch_bounds__(64) k_vk_factor(const int* __restrict__ pu_ptr, const int64_t* __restrict__ luoff,
                                                  double* __restrict__ lu, int* __restrict__ perm,
                                                  int* __restrict__ singular) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const int p0 = pu_ptr[i], m = pu_ptr[i + 1] - p0 + 1;
  double* M = lu + luoff[i];
  int* P = perm + p0 + i;
  for (int a = lane; a < m; a += 64) P[a] = a;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const double* col = M + (size_t)k * m;
    double best = -1.0;
    int bi = m;
    for (int a = k + lane; a < m; a += 64) {
      const double v = fabs(col[a]);
      if (v > best) {
        best = v;
        bi = a;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (!(best > 0.0)) {  // zero or NaN pivot column
      if (lane == 0) atomicOr(singular, 1);
      return;
    }
    const int p = bi;
    if (p != k) {
      for (int t = lane; t < m; t += 64) {
        double* ct = M + (size_t)t * m;
        const double tmp = ct[k];
        ct[k] = ct[p];
        ct[p] = tmp;
      }
      if (lane == 0) {
        const int tp = P[k];
        P[k] = P[p];
        P[p] = tp;
      }
    }
    __syncthreads();
    const double d = M[(size_t)k * m + k];
    for (int a = k + 1 + lane; a < m; a += 64) M[(size_t)k * m + a] /= d;
    __syncthreads();
    for (int a = k + 1 + lane; a < m; a += 64) {
      const double l = M[(size_t)k * m + a];
      for (int t = k + 1; t < m; ++t) M[(size_t)t * m + a] -= l * M[(size_t)t * m + k];
    }
    __syncthreads();
  }
}

// Explicit inverse of every patch's local matrix from its LU factors
// (column t of the inverse solves L U y = P e_t; one lane per column)
__global__ void __launch_bounds__(64) k_vk_invert(const int* __restrict__ pu_ptr, const int64_t* __restrict__ luoff,
                                                  const double* __restrict__ lu, const int* __restrict__ perm,
                                                  double* __restrict__ inv) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const int p0 = pu_ptr[i], m = pu_ptr[i + 1] - p0 + 1;
  const double* M = lu + luoff[i];
  double* Y = inv + luoff[i];
  const int* P = perm + p0 + i;
  for (int t = lane; t < m; t += 64) {
    double* y = Y + (size_t)t * m;
    for (int a = 0; a < m; ++a) y[a] = P[a] == t ? 1.0 : 0.0;
    for (int k = 0; k < m; ++k) {
      const double yk = y[k];
      if (yk == 0.0) continue;
      const double* ck = M + (size_t)k * m;
      for (int a = k + 1; a < m; ++a) y[a] -= ck[a] * yk;
    }
    for (int k = m - 1; k >= 0; --k) {
      const double* ck = M + (size_t)k * m;
      const double yk = y[k] / ck[k];
      y[k] = yk;
      for (int a = 0; a < k; ++a) y[a] -= ck[a] * yk;
    }
  }
}

// A colour of a sweep runs in two launches.  First the local residuals of
// all its patches at once (the rows of the colour's patches, listed patch
// after patch in `crow`; G lanes per row): rr[t] = (b - K x)[crow[t]].
template <int G>
__global__ void k_vk_colour_resid(int t0, int t1, const int* __restrict__ crow, int nu,
                                  const int* __restrict__ uu_ptr, const int* __restrict__ uu_col,
                                  const double* __restrict__ uu_val, const int* __restrict__ up_ptr,
                                  const int* __restrict__ up_col, const double* __restrict__ up_val,
                                  const int* __restrict__ pu_ptr, const int* __restrict__ pu_col,
                                  const double* __restrict__ pu_val, const int* __restrict__ c_ptr,
                                  const int* __restrict__ c_col, const double* __restrict__ c_val,
                                  const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ rr) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = t0 + (int)(q / G), g = (int)(q % G);
  if (t >= t1) return;
  const int row = crow[t];
  double s = 0.0;
  if (row < nu) {
    for (int e = uu_ptr[row] + g; e < uu_ptr[row + 1]; e += G) s += uu_val[e] * x[uu_col[e]];
    for (int e = up_ptr[row] + g; e < up_ptr[row + 1]; e += G) s += up_val[e] * x[nu + up_col[e]];
  } else {
    const int i = row - nu;
    for (int e = pu_ptr[i] + g; e < pu_ptr[i + 1]; e += G) s += pu_val[e] * x[pu_col[e]];
    for (int e = c_ptr[i] + g; e < c_ptr[i + 1]; e += G) s -= c_val[e] * x[nu + c_col[e]];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  if (g == 0) rr[t] = b[row] - s;
}

// Then the local solves (eq. locsys) with the patches' inverses and the
// relaxed updates (eq. vankasmooth).  A block takes rows 64k .. 64k+63 of the
// local solve of the patch at sweep position q (whose rows start at
// roff[q]), (q, k) from its work entry q * 32 + k; its four wavefronts split
// the columns of the inverse and add their partial sums in LDS.  Dynamic
// LDS: mmax + 256 doubles.
template <typename T>
__global__ void __launch_bounds__(256) k_vk_colour_solve(int w0, const int* __restrict__ work,
                                                         const int* __restrict__ clist,
                                                         const int* __restrict__ roff, const int* __restrict__ crow,
                                                         const double* __restrict__ rr,
                                                         const int64_t* __restrict__ luoff,
                                                         const T* __restrict__ inv, double* __restrict__ x,
                                                         double omega) {
  extern __shared__ double sh[];
  const int wv = work[w0 + blockIdx.x];
  const int q = wv >> 5, a0 = 64 * (wv & 31);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i = clist[q], r0 = roff[q], m = roff[q + 1] - r0;
  double* r = sh;
  double* part = sh + m;
  for (int t = tid; t < m; t += 256) r[t] = rr[r0 + t];
  __syncthreads();
  const T* Y = inv + luoff[i];
  const int a = a0 + lane;
  const int t0 = (w * m) >> 2, t1 = ((w + 1) * m) >> 2;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  if (a < m) {
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
      const double y0 = (double)Y[(size_t)t * m + a], y1 = (double)Y[(size_t)(t + 1) * m + a];
      const double y2 = (double)Y[(size_t)(t + 2) * m + a], y3 = (double)Y[(size_t)(t + 3) * m + a];
      d0 += y0 * r[t];
      d1 += y1 * r[t + 1];
      d2 += y2 * r[t + 2];
      d3 += y3 * r[t + 3];
    }
    for (; t < t1; ++t) d0 += (double)Y[(size_t)t * m + a] * r[t];
  }
  part[tid] = (d0 + d1) + (d2 + d3);
  __syncthreads();
  if (w == 0 && a < m) {
    const double d = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
    x[crow[r0 + a]] += omega * d;
  }
}

// Additive sweep, local solves (eq. locsys for every patch with the residual
// r of the whole level, gathered through crow; each correction goes to its
// unknown-sorted slot dpos of dd, x is not touched), one wavefront per work entry and
// four entries per block: wavefront w of block b takes entry 4b + w (rows
// 64k .. 64k+63 of its patch), gathers the patch's residual into its own LDS
// slice and sums over every column of the inverse itself (no
// cross-wavefront reduction).  Dynamic LDS: 4 * mmax doubles.
template <typename T>
__global__ void __launch_bounds__(256) k_vk_add_solve(int nw, const int* __restrict__ work, int mmax,
                                                        const int* __restrict__ clist, const int* __restrict__ roff,
                                                        const int* __restrict__ crow,
                                                        const double* __restrict__ r_all,
                                                        const int64_t* __restrict__ luoff,
                                                        const T* __restrict__ inv, const int* __restrict__ dpos,
                                                        double* __restrict__ dd) {
  extern __shared__ double sh[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = 4 * blockIdx.x + w;
  double* r = sh + (size_t)w * mmax;
  int q = 0, a0 = 0, r0 = 0, m = 0;
  if (e < nw) {
    const int wv = work[e];
    q = wv >> 5;
    a0 = 64 * (wv & 31);
    r0 = roff[q];
    m = roff[q + 1] - r0;
    for (int t = lane; t < m; t += 64) r[t] = r_all[crow[r0 + t]];
  }
  __syncthreads();
  const int a = a0 + lane;
  if (e >= nw || a >= m) return;
  const T* Y = inv + luoff[clist[q]] + a;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  int t = 0;
  for (; t + 4 <= m; t += 4) {
    d0 += (double)Y[(size_t)t * m] * r[t];
    d1 += (double)Y[(size_t)(t + 1) * m] * r[t + 1];
    d2 += (double)Y[(size_t)(t + 2) * m] * r[t + 2];
    d3 += (double)Y[(size_t)(t + 3) * m] * r[t + 3];
  }
  for (; t < m; ++t) d0 += (double)Y[(size_t)t * m] * r[t];
  dd[dpos[r0 + a]] = (d0 + d1) + (d2 + d3);
}

// Round the patch inverses to fp32 (the local solves of a precision-1
// hierarchy; round to nearest)
__global__ void k_vk_round_inv(long n, const double* __restrict__ x, float* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// Additive sweep, update: x_j += omega * (mean of the corrections of the
// patches holding unknown j), summed in patch order; an unknown in no patch
// keeps its value
__global__ void k_vk_add_gather(int n, const int* __restrict__ dptr, const double* __restrict__ dd,
                                double* __restrict__ x, double omega) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int e0 = dptr[j], e1 = dptr[j + 1];
  if (e1 == e0) return;
  double s = 0.0;
  for (int e = e0; e < e1; ++e) s += dd[e];
  x[j] += omega * (s / (double)(e1 - e0));
}

__global__ void k_vk_zero(long n, double* __restrict__ x) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = 0.0;
}

// r = b - K x on a level: rows [0, nu) use Kuu and Kup, rows [nu, nu+np) use
// Kpu and -C; G lanes per row
template <int G>
__global__ void k_vk_resid(int nu, int np, const int* __restrict__ uu_ptr, const int* __restrict__ uu_col,
                           const double* __restrict__ uu_val, const int* __restrict__ up_ptr,
                           const int* __restrict__ up_col, const double* __restrict__ up_val,
                           const int* __restrict__ pu_ptr, const int* __restrict__ pu_col,
                           const double* __restrict__ pu_val, const int* __restrict__ c_ptr,
                           const int* __restrict__ c_col, const double* __restrict__ c_val,
                           const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t / G), lane = (int)(t % G);
  if (row >= nu + np) return;
  double s = 0.0;
  if (row < nu) {
    for (int e = uu_ptr[row] + lane; e < uu_ptr[row + 1]; e += G) s += uu_val[e] * x[uu_col[e]];
    for (int e = up_ptr[row] + lane; e < up_ptr[row + 1]; e += G) s += up_val[e] * x[nu + up_col[e]];
  } else {
    const int i = row - nu;
    for (int e = pu_ptr[i] + lane; e < pu_ptr[i + 1]; e += G) s += pu_val[e] * x[pu_col[e]];
    for (int e = c_ptr[i] + lane; e < c_ptr[i + 1]; e += G) s -= c_val[e] * x[nu + c_col[e]];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  if (lane == 0) r[row] = b[row] - s;
}

// y = M x (add = 0) or y += M x (add = 1); M == nullptr stands for the identity
__global__ void k_vk_apply(int rows, const int* __restrict__ ptr, const int* __restrict__ col,
                           const double* __restrict__ val, const double* __restrict__ x, double* __restrict__ y,
                           int add) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t >> 3), lane = (int)(t & 7);
  if (row >= rows) return;
  double s = 0.0;
  if (ptr) {
    for (int e = ptr[row] + lane; e < ptr[row + 1]; e += 8) s += val[e] * x[col[e]];
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 8);
  } else {
    s = x[row];
  }
  if (lane == 0) y[row] = add ? y[row] + s : s;
}

// dense row-major copy of the coarsest coupled system [Kuu Kup; Kpu -C]
__global__ void k_vk_dense(int nu, int np, const int* __restrict__ uu_ptr, const int* __restrict__ uu_col,
                           const double* __restrict__ uu_val, const int* __restrict__ up_ptr,
                           const int* __restrict__ up_col, const double* __restrict__ up_val,
                           const int* __restrict__ pu_ptr, const int* __restrict__ pu_col,
                           const double* __restrict__ pu_val, const int* __restrict__ c_ptr,
                           const int* __restrict__ c_col, const double* __restrict__ c_val, double* __restrict__ D) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = nu + np;
  if (row >= n) return;
  double* d = D + (size_t)row * n;
  for (int t = 0; t < n; ++t) d[t] = 0.0;
  if (row < nu) {
    for (int e = uu_ptr[row]; e < uu_ptr[row + 1]; ++e) d[uu_col[e]] = uu_val[e];
    for (int e = up_ptr[row]; e < up_ptr[row + 1]; ++e) d[nu + up_col[e]] = up_val[e];
  } else {
    const int i = row - nu;
    for (int e = pu_ptr[i]; e < pu_ptr[i + 1]; ++e) d[pu_col[e]] = pu_val[e];
    for (int e = c_ptr[i]; e < c_ptr[i + 1]; ++e) d[nu + c_col[e]] = -c_val[e];
  }
}

// explicit inverse by Gauss-Jordan with partial pivoting on [D | I], one
// workgroup; D is destroyed, fcol holds the column of multipliers of a step
__global__ void __launch_bounds__(1024) k_vk_gauss_jordan(int n, double* __restrict__ D, double* __restrict__ Inv,
                                                          double* __restrict__ fcol, int* __restrict__ singular) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (size_t t = tid; t < (size_t)n * n; t += nt) Inv[t] = (t / n == t % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = n;
    for (int a = k + tid; a < n; a += nt) {
      const double v = fabs(D[(size_t)a * n + k]);
      if (v > best) {
        best = v;
        bi = a;
      }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) {
        const double ob = sv[tid + w];
        const int oi = si[tid + w];
        if (ob > sv[tid] || (ob == sv[tid] && oi < si[tid])) {
          sv[tid] = ob;
          si[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int p = si[0];
    const bool ok = sv[0] > 0.0;
    __syncthreads();
    if (!ok) {
      if (tid == 0) *singular = 1;
      return;
    }
    if (p != k)
      for (int t = tid; t < n; t += nt) {
        double u = D[(size_t)k * n + t];
        D[(size_t)k * n + t] = D[(size_t)p * n + t];
        D[(size_t)p * n + t] = u;
        u = Inv[(size_t)k * n + t];
        Inv[(size_t)k * n + t] = Inv[(size_t)p * n + t];
        Inv[(size_t)p * n + t] = u;
      }
    __syncthreads();
    const double inv_d = 1.0 / D[(size_t)k * n + k];
    __syncthreads();
    for (int t = tid; t < n; t += nt) {
      D[(size_t)k * n + t] *= inv_d;
      Inv[(size_t)k * n + t] *= inv_d;
    }
    for (int a = tid; a < n; a += nt) fcol[a] = a == k ? 0.0 : D[(size_t)a * n + k];
    __syncthreads();
    for (size_t t = tid; t < (size_t)n * n; t += nt) {
      const int a = (int)(t / n), cc = (int)(t % n);
      const double f = fcol[a];
      if (f != 0.0) {
        D[t] -= f * D[(size_t)k * n + cc];
        Inv[t] -= f * Inv[(size_t)k * n + cc];
      }
    }
    __syncthreads();
  }
}

// y = Inv b, one 64-lane wavefront per row
__global__ void k_vk_dense_mv(int n, const double* __restrict__ Inv, const double* __restrict__ b,
                              double* __restrict__ y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t >> 6), lane = (int)(t & 63);
  if (row >= n) return;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s += Inv[(size_t)row * n + c] * b[c];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[row] = s;
}

// node-interleaved r (4 per node) -> [u; p], divided by *scale if given (and
// the divided vector written to rs)
__global__ void k_vk_split(int n, const double* __restrict__ r, const double* __restrict__ scale,
                           double* __restrict__ rs, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  double v = r[t];
  if (scale) {
    v /= scale[0];
    if (rs) rs[t] = v;
  }
  const int i = t >> 2, c = t & 3;
  out[c < 3 ? 3 * i + c : 3 * n + i] = v;
}

__global__ void k_vk_join(int n, const double* __restrict__ in, double* __restrict__ z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int i = t >> 2, c = t & 3;
  z[t] = in[c < 3 ? 3 * i + c : 3 * n + i];
}

// ---------------------------------------------------------------- host code

#define VK_BLOCKS(V)                                                                                        \
  (V).Kuu->ptr.p, (V).Kuu->col.p, (V).Kuu->val.p, (V).Kup.ptr.p, (V).Kup.col.p, (V).Kup.val.p, (V).Kpu.ptr.p, \
      (V).Kpu.col.p, (V).Kpu.val.p, (V).C->ptr.p, (V).C->col.p, (V).C->val.p

void copy_async(hipStream_t s, const Csr<double>& src, Csr<double>& dst) {
  dst.rows = src.rows;
  dst.cols = src.cols;
  dst.nnz = src.nnz;
  dst.ptr.ensure(src.rows + 1);
  dst.col.ensure(src.nnz);
  dst.val.ensure(src.nnz);
  HIP_CHECK(hipMemcpyAsync(dst.ptr.p, src.ptr.p, sizeof(int) * (src.rows + 1), hipMemcpyDeviceToDevice, s));
  if (src.nnz) {
    HIP_CHECK(hipMemcpyAsync(dst.col.p, src.col.p, sizeof(int) * src.nnz, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(dst.val.p, src.val.p, sizeof(double) * src.nnz, hipMemcpyDeviceToDevice, s));
  }
}

// Build the AMG hierarchy of one block into dst with the library's set-up
// (build_levels works on the context's hierarchy: the context's own
// hierarchy is set aside meanwhile and restored on every exit).
void build_component(hfsi_ctx* c, Hierarchy& dst, const Csr<double>& A0, bool three, const hfsi_amg_params& prm) {
  Hierarchy saved;
  std::swap(c->H, saved);
  struct Restore {
    hfsi_ctx* c;
    Hierarchy& saved;
    ~Restore() { std::swap(c->H, saved); }
  } restore{c, saved};
  c->H.L.emplace_back();
  Level& L0 = c->H.L[0];
  copy_async(c->stream, A0, L0.A);
  L0.n = A0.rows;
  L0.comp.ensure(L0.n);
  k_vk_comp<<<div_up(L0.n, 256), 256, 0, c->stream>>>(L0.n, three ? 1 : 0, L0.comp.p);
  HIP_LAUNCH_CHECK();
  build_levels(c, prm, nullptr);
  std::swap(dst, c->H);  // dst takes the new hierarchy; its old one leaves with `saved`
}

// first-fit colouring of the patches on the conflict pattern G (n x n,
// structurally symmetric) plus the pattern E; returns the sweep order and
// the colour ranges
void colour_patches(const std::vector<int>& gptr, const std::vector<int>& gcol, const std::vector<int>& eptr,
                    const std::vector<int>& ecol, int n, std::vector<int>& colour, std::vector<int>& order,
                    std::vector<int>& cptr) {
  colour.assign(n, -1);
  std::vector<int> seen;  // seen[c] == i: colour c taken by a neighbour of i
  int ncol = 0;
  for (int i = 0; i < n; ++i) {
    auto mark = [&](int k) {
      if (k < i) {
        const int ck = colour[k];
        if (ck >= (int)seen.size()) seen.resize(ck + 1, -1);
        seen[ck] = i;
      }
    };
    for (int e = gptr[i]; e < gptr[i + 1]; ++e) mark(gcol[e]);
    for (int e = eptr[i]; e < eptr[i + 1]; ++e) mark(ecol[e]);
    int cc = 0;
    while (cc < (int)seen.size() && seen[cc] == i) ++cc;
    colour[i] = cc;
    ncol = std::max(ncol, cc + 1);
  }
  cptr.assign(ncol + 1, 0);
  for (int i = 0; i < n; ++i) ++cptr[colour[i] + 1];
  for (int k = 0; k < ncol; ++k) cptr[k + 1] += cptr[k];
  order.resize(n);
  std::vector<int> fill(cptr.begin(), cptr.end() - 1);
  for (int i = 0; i < n; ++i) order[fill[colour[i]]++] = i;
}

void vanka_level_data(hfsi_ctx* c, VkLevel& V, int* singular, bool additive, bool f32) {
  hipStream_t s = c->stream;
  const int np = V.np;
  // patch sizes and factor offsets
  std::vector<int> pptr = V.Kpu.ptr.download(np + 1, s);
  std::vector<int64_t> off(np);
  int64_t tot = 0;
  int mmax = 0;
  for (int i = 0; i < np; ++i) {
    const int m = pptr[i + 1] - pptr[i] + 1;
    mmax = std::max(mmax, m);
    off[i] = tot;
    tot += (int64_t)m * m;
  }
  if (mmax > kMaxPatch) fail(HFSI_E_CAPACITY, "Vanka: a patch has more than 2048 unknowns");
  if (np >= (1 << 26)) fail(HFSI_E_CAPACITY, "Vanka: more than 2^26 patches on a level");
  V.mmax = mmax;
  V.luoff.upload(off.data(), np, s);
  V.inv.ensure(tot);
  {
    DevBuf<double> lu;
    DevBuf<int> perm;
    lu.ensure(tot);
    perm.ensure((size_t)V.Kpu.nnz + np);
    k_vk_build<<<np, 64, 0, s>>>(V.nu, VK_BLOCKS(V), V.luoff.p, lu.p);
    HIP_LAUNCH_CHECK();
    k_vk_factor<<<np, 64, 0, s>>>(V.Kpu.ptr.p, V.luoff.p, lu.p, perm.p, singular);
    HIP_LAUNCH_CHECK();
    k_vk_invert<<<np, 64, 0, s>>>(V.Kpu.ptr.p, V.luoff.p, lu.p, perm.p, V.inv.p);
    HIP_LAUNCH_CHECK();
    if (f32) {
      V.inv32.ensure(tot);
      k_vk_round_inv<<<div_up(tot, 256), 256, 0, s>>>(tot, V.inv.p, V.inv32.p);
      HIP_LAUNCH_CHECK();
    } else {
      V.inv32.release();
    }
  }
  // lanes per row of the sweep's residual, from the average row length
  const double avg = (double)(V.Kuu->nnz + V.Kup.nnz + V.Kpu.nnz + V.C->nnz) / (double)(V.nu + V.np);
  V.lanes = avg <= 48 ? 8 : (avg <= 96 ? 16 : (avg <= 192 ? 32 : 64));
  std::vector<int> colour, order;
  if (additive) {  // no order: the patches by index, one range
    colour.assign(np, 0);
    order.resize(np);
    for (int i = 0; i < np; ++i) order[i] = i;
    V.cptr = {0, np};
  } else {
    // conflict pattern B2 A B1^T (+ C) and the colours
    DevBuf<int> flags;
    flags.zero(1, s);
    Csr<double> T, G;
    sparse_product(c, V.Kpu, *V.Kuu, T, flags.p);
    sparse_product(c, T, V.Kup, G, flags.p);
    std::vector<int> gptr = G.ptr.download(np + 1, s);
    std::vector<int> gcol = G.col.download(G.nnz, s);
    std::vector<int> eptr = V.C->ptr.download(np + 1, s);
    std::vector<int> ecol = V.C->col.download(V.C->nnz, s);
    int fl = 0;
    HIP_CHECK(hipMemcpyAsync(&fl, flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (fl) fail(HFSI_E_CAPACITY, "Vanka: conflict pattern product overflowed");
    colour_patches(gptr, gcol, eptr, ecol, np, colour, order, V.cptr);
  }
  // the patches' rows in sweep order (displacement unknowns, then the pressure)
  std::vector<int> pcol = V.Kpu.col.download(V.Kpu.nnz, s);
  V.hroff.assign(np + 1, 0);
  std::vector<int> crow;
  crow.reserve((size_t)V.Kpu.nnz + np);
  for (int q = 0; q < np; ++q) {
    const int i = order[q];
    for (int e = pptr[i]; e < pptr[i + 1]; ++e) crow.push_back(pcol[e]);
    crow.push_back(V.nu + i);
    V.hroff[q + 1] = (int)crow.size();
  }
  V.crow.upload(crow.data(), crow.size(), s);
  V.roff.upload(V.hroff.data(), np + 1, s);
  {
    std::vector<int> work;
    V.hwptr.assign(V.cptr.size(), 0);
    for (size_t k = 0; k + 1 < V.cptr.size(); ++k) {
      V.hwptr[k] = (int)work.size();
      for (int q = V.cptr[k]; q < V.cptr[k + 1]; ++q)
        for (int a0 = 0; a0 < V.hroff[q + 1] - V.hroff[q]; a0 += 64) work.push_back(q * 32 + a0 / 64);
    }
    V.hwptr.back() = (int)work.size();
    V.work.upload(work.data(), work.size(), s);
    HIP_CHECK(hipStreamSynchronize(s));  // the host list leaves scope
  }
  V.clist.upload(order.data(), np, s);
  V.colour.upload(colour.data(), np, s);
  std::vector<int> dptr, dpos;
  if (additive) {
    // unknown -> its entries of crow, in increasing entry (= patch) order
    const int n = V.nu + np;
    dptr.assign(n + 1, 0);
    for (int row : crow) ++dptr[row + 1];
    for (int j = 0; j < n; ++j) dptr[j + 1] += dptr[j];
    dpos.resize(crow.size());
    std::vector<int> fill(dptr.begin(), dptr.end() - 1);
    for (size_t e = 0; e < crow.size(); ++e) dpos[e] = fill[crow[e]]++;
    V.dptr.upload(dptr.data(), n + 1, s);
    V.dpos.upload(dpos.data(), dpos.size(), s);
    V.dd.ensure(crow.size());
  } else {
    V.rr.ensure(crow.size());
  }
  HIP_CHECK(hipStreamSynchronize(s));  // the host vectors leave scope
  if (f32) V.inv.release();            // the sweeps read inv32 only
}

template <int G>
void sweep_g(hipStream_t s, VkLevel& V, const double* b, double* x, double omega) {
  const size_t lds = sizeof(double) * (V.mmax + 256);
  for (size_t k = 0; k + 1 < V.cptr.size(); ++k) {
    const int q0 = V.cptr[k], q1 = V.cptr[k + 1];
    if (q1 == q0) continue;
    const int t0 = V.hroff[q0], t1 = V.hroff[q1];
    const int w0 = V.hwptr[k], nw = V.hwptr[k + 1] - w0;
    k_vk_colour_resid<G><<<div_up((long)(t1 - t0) * G, 256), 256, 0, s>>>(t0, t1, V.crow.p, V.nu, VK_BLOCKS(V), b, x,
                                                                          V.rr.p);
    if (V.inv32.p)
      k_vk_colour_solve<float><<<nw, 256, lds, s>>>(w0, V.work.p, V.clist.p, V.roff.p, V.crow.p, V.rr.p, V.luoff.p,
                                                    V.inv32.p, x, omega);
    else
      k_vk_colour_solve<double><<<nw, 256, lds, s>>>(w0, V.work.p, V.clist.p, V.roff.p, V.crow.p, V.rr.p, V.luoff.p,
                                                     V.inv.p, x, omega);
  }
  HIP_LAUNCH_CHECK();
}

// additive sweep: residual of x on the whole level, every local solve, the
// averaged update
template <int G>
void sweep_additive_g(hipStream_t s, VkLevel& V, const double* b, double* x, double omega) {
  const int n = V.nu + V.np;
  k_vk_resid<G><<<div_up((long)n * G, 256), 256, 0, s>>>(V.nu, V.np, VK_BLOCKS(V), b, x, V.r.p);
  const int nw = V.hwptr.back();
  const size_t lds4 = sizeof(double) * 4 * (size_t)V.mmax;
  if (V.inv32.p)
    k_vk_add_solve<float><<<div_up(nw, 4), 256, lds4, s>>>(nw, V.work.p, V.mmax, V.clist.p, V.roff.p, V.crow.p,
                                                              V.r.p, V.luoff.p, V.inv32.p, V.dpos.p, V.dd.p);
  else
    k_vk_add_solve<double><<<div_up(nw, 4), 256, lds4, s>>>(nw, V.work.p, V.mmax, V.clist.p, V.roff.p, V.crow.p,
                                                               V.r.p, V.luoff.p, V.inv.p, V.dpos.p, V.dd.p);
  k_vk_add_gather<<<div_up(n, 256), 256, 0, s>>>(n, V.dptr.p, V.dd.p, x, omega);
  HIP_LAUNCH_CHECK();
}

void sweep(hipStream_t s, VkLevel& V, const double* b, double* x, double omega, bool additive) {
  if (additive) {
    switch (V.lanes) {
      case 8: sweep_additive_g<8>(s, V, b, x, omega); break;
      case 16: sweep_additive_g<16>(s, V, b, x, omega); break;
      case 32: sweep_additive_g<32>(s, V, b, x, omega); break;
      default: sweep_additive_g<64>(s, V, b, x, omega); break;
    }
    return;
  }
  switch (V.lanes) {
    case 8: sweep_g<8>(s, V, b, x, omega); break;
    case 16: sweep_g<16>(s, V, b, x, omega); break;
    case 32: sweep_g<32>(s, V, b, x, omega); break;
    default: sweep_g<64>(s, V, b, x, omega); break;
  }
}

void apply_block(hipStream_t s, int rows, const Csr<double>* M, const double* x, double* y, bool add) {
  k_vk_apply<<<div_up((long)rows * 8, 256), 256, 0, s>>>(rows, M ? M->ptr.p : nullptr, M ? M->col.p : nullptr,
                                                          M ? M->val.p : nullptr, x, y, add ? 1 : 0);
  HIP_LAUNCH_CHECK();
}

// x_l = V-cycle applied to b_l (zero start)
// kernel launches only (no allocation, copy or synchronisation): the cycle is
// captured into a graph once per set-up
void cycle(hipStream_t s, Coupled& V, int l) {
  VkLevel& L = V.L[l];
  const int n = L.nu + L.np;
  if (l + 1 == (int)V.L.size()) {
    k_vk_dense_mv<<<div_up((long)n * 64, 256), 256, 0, s>>>(n, V.cinv.p, L.b.p, L.x.p);
    HIP_LAUNCH_CHECK();
    return;
  }
  k_vk_zero<<<div_up(n, 256), 256, 0, s>>>(n, L.x.p);
  for (int k = 0; k < V.steps; ++k) sweep(s, L, L.b.p, L.x.p, V.omega, V.additive);
  k_vk_resid<8><<<div_up((long)n * 8, 256), 256, 0, s>>>(L.nu, L.np, VK_BLOCKS(L), L.b.p, L.x.p, L.r.p);
  HIP_LAUNCH_CHECK();
  VkLevel& N = V.L[l + 1];
  apply_block(s, N.nu, L.Ru, L.r.p, N.b.p, false);
  apply_block(s, N.np, L.Rp, L.r.p + L.nu, N.b.p + N.nu, false);
  cycle(s, V, l + 1);
  apply_block(s, L.nu, L.Pu, N.x.p, L.x.p, true);
  apply_block(s, L.np, L.Pp, N.x.p + N.nu, L.x.p + L.nu, true);
  for (int k = 0; k < V.steps; ++k) sweep(s, L, L.b.p, L.x.p, V.omega, V.additive);
}

}  // namespace

void vanka_free(hfsi_ctx* c) {
  delete reinterpret_cast<Coupled*>(c->vanka_impl);
  c->vanka_impl = nullptr;
}

void vanka_invalidate(hfsi_ctx* c) {
  if (c->vanka_impl) reinterpret_cast<Coupled*>(c->vanka_impl)->ready = false;
  c->precond_kind = 0;
  c->keep_valid = false;
}

void vanka_setup(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info) {
  hipStream_t s = c->stream;
  if (c->A.rows != 3 * c->n) fail(HFSI_E_ORDER, "coupled AMG: needs the assembled tangent");
  if (prm.interp != 0) fail(HFSI_E_ARG, "coupled AMG: interp must be 0 (no learned interpolation)");
  if (prm.drop_tol != 0.0) fail(HFSI_E_ARG, "coupled AMG: drop_tol must be 0");
  HIP_CHECK(hipEventRecord(c->ev0, s));
  c->precond_kind = 0;
  Coupled& V = state(c);
  V.ready = false;
  V.drop_graph();
  V.L.clear();
  V.omega = prm.vanka_omega;
  V.steps = prm.vanka_steps;
  V.additive = prm.coupled == 2;
  hfsi_amg_params cp = prm;
  cp.smoother = 0;  // the component hierarchies give only P; their smoother data is unused
  cp.precision = 0;
  // level-0 blocks
  const int n = c->n;
  VkLevel L0;
  Csr<double> C0;
  L0.Kup.rows = 3 * n;
  L0.Kup.cols = n;
  L0.Kup.nnz = 3L * c->nb;
  L0.Kpu.rows = n;
  L0.Kpu.cols = 3 * n;
  L0.Kpu.nnz = 3L * c->nb;
  C0.rows = C0.cols = n;
  C0.nnz = c->nb;
  L0.Kup.ptr.ensure(3 * n + 1);
  L0.Kup.col.ensure(3L * c->nb);
  L0.Kup.val.ensure(3L * c->nb);
  L0.Kpu.ptr.ensure(n + 1);
  L0.Kpu.col.ensure(3L * c->nb);
  L0.Kpu.val.ensure(3L * c->nb);
  C0.ptr.ensure(n + 1);
  C0.col.ensure(c->nb);
  C0.val.ensure(c->nb);
  k_vk_ptr0<<<div_up(n + 1, 256), 256, 0, s>>>(n, c->nptr.p, L0.Kup.ptr.p, L0.Kpu.ptr.p, C0.ptr.p);
  k_vk_blocks0<<<div_up(c->nb, 256), 256, 0, s>>>(c->nb, c->brow.p, c->nptr.p, c->ncol.p, c->Kval.p, L0.Kup.col.p,
                                                 L0.Kup.val.p, L0.Kpu.col.p, L0.Kpu.val.p, C0.col.p, C0.val.p);
  HIP_LAUNCH_CHECK();
  build_component(c, V.Hu, c->A, true, cp);
  build_component(c, V.Hp, C0, false, cp);
  const int lu = (int)V.Hu.L.size(), lp = (int)V.Hp.L.size();
  const int nl = std::max(lu, lp);
  V.L.resize(nl);
  V.L[0].Kup = std::move(L0.Kup);
  V.L[0].Kpu = std::move(L0.Kpu);
  for (int l = 0; l < nl; ++l) {
    VkLevel& L = V.L[l];
    L.Kuu = &V.Hu.L[std::min(l, lu - 1)].A;
    L.C = &V.Hp.L[std::min(l, lp - 1)].A;
    L.nu = L.Kuu->rows;
    L.np = L.C->rows;
    if (l + 1 < nl) {
      if (l + 1 < lu) {
        L.Pu = &V.Hu.L[l].P;
        L.Ru = &V.Hu.L[l].R;
      }
      if (l + 1 < lp) {
        L.Pp = &V.Hp.L[l].P;
        L.Rp = &V.Hp.L[l].R;
      }
    }
  }
  // coarse B blocks: Kup' = Ru Kup Pp, Kpu' = Rp Kpu Pu
  DevBuf<int> flags;
  flags.zero(1, s);
  for (int l = 0; l + 1 < nl; ++l) {
    VkLevel& L = V.L[l];
    VkLevel& N = V.L[l + 1];
    Csr<double> T;
    if (L.Pp) sparse_product(c, L.Kup, *L.Pp, T, flags.p);
    else copy_async(s, L.Kup, T);
    if (L.Ru) sparse_product(c, *L.Ru, T, N.Kup, flags.p);
    else N.Kup = std::move(T);
    Csr<double> T2;
    if (L.Pu) sparse_product(c, L.Kpu, *L.Pu, T2, flags.p);
    else copy_async(s, L.Kpu, T2);
    if (L.Rp) sparse_product(c, *L.Rp, T2, N.Kpu, flags.p);
    else N.Kpu = std::move(T2);
  }
  int fl = 0;
  HIP_CHECK(hipMemcpyAsync(&fl, flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (fl) fail(HFSI_E_CAPACITY, "coupled AMG: a coarse block product overflowed");
  // smoother data, vectors
  DevBuf<int> singular;
  singular.zero(1, s);
  for (int l = 0; l < nl; ++l) {
    VkLevel& L = V.L[l];
    const size_t n_l = (size_t)L.nu + L.np;
    L.x.ensure(n_l);
    L.b.ensure(n_l);
    L.r.ensure(n_l);
    if (l + 1 < nl) vanka_level_data(c, L, singular.p, V.additive, prm.precision == 1);
  }
  // coarsest: explicit inverse
  VkLevel& Lc = V.L.back();
  const int nc = Lc.nu + Lc.np;
  if (nc > kMaxCoarsest) fail(HFSI_E_CAPACITY, "coupled AMG: coarsest system larger than 4096 unknowns");
  V.nc = nc;
  {
    DevBuf<double> D, fcol;
    D.ensure((size_t)nc * nc);
    fcol.ensure(nc);
    V.cinv.ensure((size_t)nc * nc);
    k_vk_dense<<<div_up(nc, 256), 256, 0, s>>>(Lc.nu, Lc.np, VK_BLOCKS(Lc), D.p);
    HIP_LAUNCH_CHECK();
    k_vk_gauss_jordan<<<1, 1024, 0, s>>>(nc, D.p, V.cinv.p, fcol.p, singular.p + 0);
    HIP_LAUNCH_CHECK();
    int sg = 0;
    HIP_CHECK(hipMemcpyAsync(&sg, singular.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (sg) fail(HFSI_E_BREAKDOWN, "coupled AMG: a local Vanka system or the coarsest system is singular");
  }
  // capture the cycle on a private stream (the context's may be the null
  // stream, which cannot be captured); replays run on the context's stream
  {
    hipStream_t cs = nullptr;
    HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{cs};
    HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      cycle(cs, V, 0);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIP_CHECK(hipStreamEndCapture(cs, &V.graph));
    HIP_CHECK(hipGraphInstantiate(&V.exec, V.graph, nullptr, nullptr, 0));
  }
  V.ready = true;
  c->precond_kind = 1;
  HIP_CHECK(hipEventRecord(c->ev1, s));
  if (info) {
    info->levels = nl;
    double nnz0 = 0, rows0 = 0, sn = 0, sr = 0;
    for (int l = 0; l < nl && l < 32; ++l) {
      const VkLevel& L = V.L[l];
      const int64_t z = L.Kuu->nnz + L.Kup.nnz + L.Kpu.nnz + L.C->nnz;
      info->rows[l] = L.nu + L.np;
      info->nnz[l] = z;
      if (l == 0) {
        nnz0 = (double)z;
        rows0 = L.nu + L.np;
      }
      sn += (double)z;
      sr += L.nu + L.np;
    }
    info->op_complexity = sn / nnz0;
    info->grid_complexity = sr / rows0;
    info->pmis_rounds = 0;
    info->rho = -1.0;
    info->rho_classical = -1.0;
    info->krylov_rho = -1.0;
    info->krylov_rho_classical = -1.0;
    info->learned_used = 0;
    info->seconds = elapsed_ms(c) * 1e-3;
  }
}

// z = V-cycle of the coupled hierarchy applied to r (node-interleaved)
void vanka_precond(hfsi_ctx* c, const double* r, double* z, const double* scale, double* rs) {
  Coupled& V = state(c);
  if (!V.ready) fail(HFSI_E_ORDER, "preconditioner: no coupled AMG hierarchy");
  hipStream_t s = c->stream;
  const int n = c->n;
  VkLevel& L0 = V.L[0];
  if (L0.np != n || L0.nu != 3 * n) fail(HFSI_E_ORDER, "preconditioner: coupled hierarchy of another mesh");
  k_vk_split<<<div_up(4L * n, 256), 256, 0, s>>>(n, r, scale, scale ? rs : nullptr, L0.b.p);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipGraphLaunch(V.exec, s));
  k_vk_join<<<div_up(4L * n, 256), 256, 0, s>>>(n, L0.x.p, z);
  HIP_LAUNCH_CHECK();
}

// host copies for inspection: which 10 = Kuu, 11 = Kup, 12 = Kpu, 13 = Kpp
// (= -C), 14 = patch colours (int32 per pressure unknown, in col), 15 = P_u,
// 16 = P_p (which 15 / 16 on a level whose transfer is the identity, 14-16 on
// the coarsest level and 14 of the additive variant are HFSI_E_ARG)
void vanka_export(hfsi_ctx* c, int level, int which, int32_t* rows, int32_t* cols, int64_t* nnz, int32_t* ptr,
                  int32_t* col, double* val) {
  if (!c->vanka_impl || !state(c).ready) fail(HFSI_E_ORDER, "amg_export: no coupled hierarchy");
  Coupled& V = state(c);
  if (level < 0 || level >= (int)V.L.size()) fail(HFSI_E_ARG, "amg_export: level out of range");
  VkLevel& L = V.L[level];
  const bool last = level + 1 == (int)V.L.size();
  hipStream_t s = c->stream;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  };
  if (which == 14) {
    if (last) fail(HFSI_E_ARG, "amg_export: the coarsest level has no patches");
    if (V.additive) fail(HFSI_E_ARG, "amg_export: the additive variant has no colours");
    if (rows) *rows = L.np;
    if (cols) *cols = (int)L.cptr.size() - 1;
    if (nnz) *nnz = L.np;
    cp(col, L.colour.p, sizeof(int) * L.np);
  } else {
    const Csr<double>* M = nullptr;
    if (which == 10) M = L.Kuu;
    else if (which == 11) M = &L.Kup;
    else if (which == 12) M = &L.Kpu;
    else if (which == 13) M = L.C;
    else if (which == 15) M = last ? nullptr : L.Pu;
    else if (which == 16) M = last ? nullptr : L.Pp;
    else fail(HFSI_E_ARG, "amg_export: unknown item");
    if (!M) fail(HFSI_E_ARG, "amg_export: identity transfer or coarsest level");
    if (rows) *rows = M->rows;
    if (cols) *cols = M->cols;
    if (nnz) *nnz = M->nnz;
    cp(ptr, M->ptr.p, sizeof(int) * (M->rows + 1));
    cp(col, M->col.p, sizeof(int) * M->nnz);
    if (val) {
      cp(val, M->val.p, sizeof(double) * M->nnz);
      if (which == 13) {
        HIP_CHECK(hipStreamSynchronize(s));
        for (int64_t e = 0; e < M->nnz; ++e) val[e] = -val[e];
      }
    }
  }
  HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace hfsi
