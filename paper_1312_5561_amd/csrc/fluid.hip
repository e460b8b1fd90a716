// The fluid sub-problem and the partitioned coupling (sections "The fluid
// sub-problem", "Stabilization for the fluid sub-problem", "A
// Dirichlet-Neumann FSI iteration" and "Aitken relaxation").
//
// A context switched to the fluid (hfsi_set_fluid) assembles, on the mesh
// moved by the mesh displacement d_f, the implicit-Euler step of the ALE
// Navier-Stokes equations with SUPG/PSPG stabilisation (eq. nstdis,
// eq. weakns, eq. stabweakfluid) into the same 4x4 node blocks as the
// structure; per tetrahedron, with c = u - w the convective velocity,
// r = (u - u_old)/dt + (c . grad) u + grad p / rho the strong momentum
// residual per unit mass and one tau = ((2/dt)^2 + (2|c_mean|/h)^2 +
// (4 nu/h^2)^2)^(-1/2):
//   R^u_a = int rho (u - u_old)/dt N_a + rho (c . grad) u N_a
//           + mu V (grad u + grad u^T) G_a - V pbar G_a + rho tau int (c . G_a) r
//   R^p_a = -V/4 div u - tau int G_a . r
// integrated by the 4-point degree-2 rule (exact here), with the exact
// Jacobian at fixed tau.  The inlet traction enters as the context's nodal
// load (hfsi_set_bc triangles, scaled by the load factor).  The Schur
// diagonal of P_L becomes s_i = C_ii + sum_j B2_ij B1^T_ji / A_jj (the
// diagonal of B2 diag(A)^-1 B1^T + C) of every assembled Jacobian.
//
// A context switched to the mesh Laplacian (hfsi_set_mesh_laplace)
// assembles the P1 Laplacian of its reference mesh on every displacement
// component (eq. harext); with every boundary node and every pressure fixed,
// one Newton step from a state holding the boundary values is the harmonic
// extension.
//
// hfsi_fsi_time_step runs the Dirichlet-Neumann iteration with Aitken
// relaxation over a fluid, a mesh and a structure context.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"

using namespace hfsi;

namespace {

constexpr double kQA = 0.5854101966249685;  // 4-point rule: barycentric (A, B, B, B)
constexpr double kQB = 0.1381966011250105;

__device__ __forceinline__ double qn(int q, int a) { return q == a ? kQA : kQB; }

// Element residual and Jacobian of the fluid step; one thread per element
// of one colour.
__global__ void __launch_bounds__(128)
k_fluid_element(int e0, int e1, int m, const int* __restrict__ T, const double* __restrict__ X,
                const double* __restrict__ dmesh, const double* __restrict__ V0s, const int* __restrict__ slot,
                const double* __restrict__ v, const double* __restrict__ uo, const double* __restrict__ wm,
                double rho, double mu, double dt, int oseen, double* __restrict__ R, double* __restrict__ Kval,
                int want_K, unsigned long long* __restrict__ minJ, int* __restrict__ inverted) {
  const int e = e0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  int nd[4];
  double x[4][3], u[4][3], p[4], c[4][3], uold[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nd[a] = T[a * m + e];
    const int k = nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x[a][i] = X[3 * k + i] + dmesh[3 * k + i];
      u[a][i] = v[4 * k + i];
      uold[a][i] = uo[3 * k + i];
      c[a][i] = (oseen ? uold[a][i] : u[a][i]) - wm[3 * k + i];
    }
    p[a] = v[4 * k + 3];
  }
  // geometry of the current tetrahedron: D = [x1-x0, x2-x0, x3-x0] (columns),
  // grad N_a = row a-1 of D^-1, grad N_0 = -(sum of the others)
  double D[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) D[i][k] = x[k + 1][i] - x[0][i];
  const double a00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double a01 = D[0][2] * D[2][1] - D[0][1] * D[2][2];
  const double a02 = D[0][1] * D[1][2] - D[0][2] * D[1][1];
  const double det = D[0][0] * a00 + D[1][0] * a01 + D[2][0] * a02;
  const double V = det / 6.0;
  const double J = V / V0s[e];
  if (!(J > 0.0)) {
    atomicMin(inverted, e);
    return;
  }
  const unsigned long long jbits = (unsigned long long)__double_as_longlong(J);
  if (jbits < __hip_atomic_load(minJ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(minJ, jbits);
  const double id = 1.0 / det;
  double G[4][3];
  // row r of D^-1 holds the cofactors of column r of D, divided by det
  G[1][0] = a00 * id;
  G[1][1] = a01 * id;
  G[1][2] = a02 * id;
  G[2][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) * id;
  G[2][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
  G[2][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
  G[3][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) * id;
  G[3][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
  G[3][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
#pragma unroll
  for (int j = 0; j < 3; ++j) G[0][j] = -(G[1][j] + G[2][j] + G[3][j]);
  double h2 = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b) {
      const double dx = x[a][0] - x[b][0], dy = x[a][1] - x[b][1], dz = x[a][2] - x[b][2];
      h2 = fmax(h2, dx * dx + dy * dy + dz * dz);
    }
  const double h = sqrt(h2);
  double cm[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) cm[i] = 0.25 * (c[0][i] + c[1][i] + c[2][i] + c[3][i]);
  const double nu = mu / rho;
  const double cn = sqrt(cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2]);
  const double t1 = 2.0 / dt, t2 = 2.0 * cn / h, t3 = 4.0 * nu / h2;
  const double tau = 1.0 / sqrt(t1 * t1 + t2 * t2 + t3 * t3);
  // gradients
  double Gu[3][3], gp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Gu[i][j] = u[0][i] * G[0][j] + u[1][i] * G[1][j] + u[2][i] * G[2][j] + u[3][i] * G[3][j];
#pragma unroll
  for (int j = 0; j < 3; ++j) gp[j] = p[0] * G[0][j] + p[1] * G[1][j] + p[2] * G[2][j] + p[3] * G[3][j];
  const double div = Gu[0][0] + Gu[1][1] + Gu[2][2];
  const double w = 0.25 * V;
  // quadrature-point values: galerkin momentum density g(q) (per unit
  // mass), strong residual r(q), c(q) . G_a
  double gq[4][3], rq[4][3], cG[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double uq[3], cq[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uq[i] = qn(q, 0) * (u[0][i] - uold[0][i]) + qn(q, 1) * (u[1][i] - uold[1][i]) +
              qn(q, 2) * (u[2][i] - uold[2][i]) + qn(q, 3) * (u[3][i] - uold[3][i]);
      cq[i] = qn(q, 0) * c[0][i] + qn(q, 1) * c[1][i] + qn(q, 2) * c[2][i] + qn(q, 3) * c[3][i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double conv = Gu[i][0] * cq[0] + Gu[i][1] * cq[1] + Gu[i][2] * cq[2];
      gq[q][i] = uq[i] / dt + conv;
      rq[q][i] = gq[q][i] + gp[i] / rho;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) cG[q][a] = cq[0] * G[a][0] + cq[1] * G[a][1] + cq[2] * G[a][2];
  }
  const double pbar = 0.25 * (p[0] + p[1] + p[2] + p[3]);
  // residual
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double* Ra = R + 4 * nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double gal = 0.0, supg = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gal += qn(q, a) * gq[q][i];
        supg += cG[q][a] * rq[q][i];
      }
      const double visc = (Gu[i][0] + Gu[0][i]) * G[a][0] + (Gu[i][1] + Gu[1][i]) * G[a][1] +
                          (Gu[i][2] + Gu[2][i]) * G[a][2];
      Ra[i] += w * rho * gal + mu * V * visc - V * pbar * G[a][i] + w * rho * tau * supg;
    }
    double pspg = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) pspg += G[a][0] * rq[q][0] + G[a][1] * rq[q][1] + G[a][2] * rq[q][2];
    Ra[3] += -w * div - w * tau * pspg;
  }
  if (!want_K) return;
  // derivative of the convective velocity c by u: 1 (Navier-Stokes), 0 (Oseen)
  const double dc = oseen ? 0.0 : 1.0;
  // per-node sums over the quadrature points
  double scG[4];  // sum_q c(q).G_a
#pragma unroll
  for (int a = 0; a < 4; ++a) scG[a] = cG[0][a] + cG[1][a] + cG[2][a] + cG[3][a];
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    double GaGu[3];  // (G_a^T Gu)_k
#pragma unroll
    for (int k = 0; k < 3; ++k) GaGu[k] = G[a][0] * Gu[0][k] + G[a][1] * Gu[1][k] + G[a][2] * Gu[2][k];
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      double NN = 0.0, NcGb = 0.0, cGdr = 0.0, cGN = 0.0, sdr = 0.0;
      double rN[3] = {0.0, 0.0, 0.0};  // sum_q N_b(q) r_i(q)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double na = qn(q, a), nb = qn(q, b);
        const double dr = nb / dt + cG[q][b];
        NN += na * nb;
        NcGb += na * cG[q][b];
        cGdr += cG[q][a] * dr;
        cGN += cG[q][a] * nb;
        sdr += dr;
#pragma unroll
        for (int i = 0; i < 3; ++i) rN[i] += nb * rq[q][i];
      }
      const double GG = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
      double blk[16];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double val = dc * w * rho * NN * Gu[i][k] + mu * V * G[a][k] * G[b][i] +
                       dc * w * rho * tau * (G[a][k] * rN[i] + cGN * Gu[i][k]);
          if (i == k) val += w * rho * (NN / dt + NcGb) + mu * V * GG + w * rho * tau * cGdr;
          blk[i * 4 + k] = val;
        }
        blk[i * 4 + 3] = -0.25 * V * G[a][i] + w * tau * scG[a] * G[b][i];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) blk[12 + k] = -w * G[b][k] - w * tau * (G[a][k] * sdr + dc * GaGu[k]);
      blk[15] = -(V * tau / rho) * GG;
      double* dst = Kval + 16 * (size_t)slot[(a * 4 + b) * m + e];
#pragma unroll
      for (int q = 0; q < 16; q += 2) {
        double2 o = *reinterpret_cast<double2*>(dst + q);
        o.x += blk[q];
        o.y += blk[q + 1];
        *reinterpret_cast<double2*>(dst + q) = o;
      }
    }
  }
}

// P1 Laplacian of the reference mesh on each displacement component:
// A_ab = V (G_a . G_b) I, R^u_a = sum_b A_ab d_b (pressure rows untouched)
__global__ void __launch_bounds__(128)
k_laplace_element(int e0, int e1, int m, const int* __restrict__ T, const double* __restrict__ Gs,
                  const double* __restrict__ Vs, const int* __restrict__ slot, const double* __restrict__ v,
                  double* __restrict__ R, double* __restrict__ Kval, int want_K) {
  const int e = e0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  int nd[4];
  double G[4][3], d[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nd[a] = T[a * m + e];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      G[a][j] = Gs[(a * 3 + j) * m + e];
      d[a][j] = v[4 * nd[a] + j];
    }
  }
  const double V = Vs[e];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double Kab[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) Kab[b] = V * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
    double* Ra = R + 4 * nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i) Ra[i] += Kab[0] * d[0][i] + Kab[1] * d[1][i] + Kab[2] * d[2][i] + Kab[3] * d[3][i];
    if (!want_K) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double* dst = Kval + 16 * (size_t)slot[(a * 4 + b) * m + e];
      dst[0] += Kab[b];
      dst[5] += Kab[b];
      dst[10] += Kab[b];
    }
  }
}

// block (j, i) of row j (columns sorted within a row), -1 if absent
__device__ int find_block(const int* __restrict__ nptr, const int* __restrict__ ncol, int j, int i) {
  int lo = nptr[j], hi = nptr[j + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ncol[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  return lo < nptr[j + 1] && ncol[lo] == i ? lo : -1;
}

// s_i = C_ii + sum_(j,c) B2_(i,jc) B1^T_(jc,i) / A_(jc,jc) on the Dirichlet-
// eliminated blocks (a fixed velocity dof has zero couplings)
__global__ void k_fluid_schur(int n, const int* __restrict__ nptr, const int* __restrict__ ncol,
                              const int* __restrict__ diag_blk, const double* __restrict__ Kval,
                              double* __restrict__ s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = -Kval[16 * (size_t)diag_blk[i] + 15];
  for (int q = nptr[i]; q < nptr[i + 1]; ++q) {
    const int j = ncol[q];
    const int qt = find_block(nptr, ncol, j, i);
    if (qt < 0) continue;
    const double* bij = Kval + 16 * (size_t)q;
    const double* bji = Kval + 16 * (size_t)qt;
    const double* bjj = Kval + 16 * (size_t)diag_blk[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double ajj = bjj[5 * c];
      if (ajj != 0.0) acc += bij[12 + c] * bji[4 * c + 3] / ajj;
    }
  }
  s[i] = acc;
}

__global__ void k_fill(long n, double value, double* __restrict__ x) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = value;
}

// ---------------------------------------------------------- FSI helpers

// the first interface displacement of a step: dG[k] = vs[4 idx[k/3] + k%3]
// + dt vel[3 idx[k/3] + k%3] (extrapolation with the structure's velocity)
__global__ void k_predict(int cnt, const int* __restrict__ idx, const double* __restrict__ vs,
                          const double* __restrict__ vel, double dt, double* __restrict__ dG) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  const int k = idx[t / 3], c = t % 3;
  dG[t] = vs[4 * k + c] + dt * vel[3 * k + c];
}

// dst[4 idx[k/3] + k%3] = src[k]
__global__ void k_scatter_u(int cnt, const int* __restrict__ idx, const double* __restrict__ src,
                            double* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  dst[4 * idx[t / 3] + t % 3] = src[t];
}

// u part of a node-interleaved vector -> [n][3]
__global__ void k_u_of(int n, const double* __restrict__ v, double* __restrict__ u) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  u[t] = v[4 * (t / 3) + t % 3];
}

// mesh displacement d = vm[:, 0:3] and velocity w = (d - d_prev) / dt
__global__ void k_mesh_motion(int n, const double* __restrict__ vm, const double* __restrict__ dprev, double dt,
                              double* __restrict__ d, double* __restrict__ wv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const double x = vm[4 * (t / 3) + t % 3];
  d[t] = x;
  wv[t] = (x - dprev[t]) / dt;
}

// the fluid's force on the wall: f[k] = -R[4 idx[k/3] + k%3], and the
// structure's nodal load: fext = 0, then fext[3 sidx[k/3] + k%3] = f[k]
__global__ void k_force(int cnt, const int* __restrict__ fidx, const double* __restrict__ R,
                        double* __restrict__ f) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  f[t] = -R[4 * fidx[t / 3] + t % 3];
}

__global__ void k_load_scatter(int cnt, const int* __restrict__ sidx, const double* __restrict__ f,
                               double* __restrict__ fext) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  fext[3 * sidx[t / 3] + t % 3] = f[t];
}

// r = s[4 sidx[k/3] + k%3] - dG[k]
__global__ void k_iface_residual(int cnt, const int* __restrict__ sidx, const double* __restrict__ vs,
                                 const double* __restrict__ dG, double* __restrict__ r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  r[t] = vs[4 * sidx[t / 3] + t % 3] - dG[t];
}

// three dot products of the interface vectors in one workgroup:
// out = (r.r, rp.(r - rp), (r - rp).(r - rp)), summed in a fixed order
__global__ void __launch_bounds__(256) k_iface_dots(int len, const double* __restrict__ r,
                                                    const double* __restrict__ rp, double* __restrict__ out) {
  __shared__ double sh[3][256];
  double a = 0.0, b = 0.0, cc = 0.0;
  for (int t = threadIdx.x; t < len; t += 256) {
    const double x = r[t];
    a += x * x;
    if (rp) {
      const double d = x - rp[t];
      b += rp[t] * d;
      cc += d * d;
    }
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = cc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = sh[threadIdx.x][0];
}

// dG += omega r; rp = r
__global__ void k_relax(int len, double omega, const double* __restrict__ r, double* __restrict__ dG,
                        double* __restrict__ rp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  dG[t] += omega * r[t];
  rp[t] = r[t];
}

// vf[4 idx[k] + c] = w[3 idx[k] + c]: the mesh velocity as the fluid's
// velocity on the interface nodes
__global__ void k_set_iface_velocity(int cnt, const int* __restrict__ idx, const double* __restrict__ wv,
                                     double* __restrict__ vf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * cnt) return;
  const int k = idx[t / 3], c = t % 3;
  vf[4 * k + c] = wv[3 * k + c];
}

__global__ void k_flags(int* inverted, unsigned long long* minJ) {
  *inverted = INT32_MAX;
  *minJ = 0x7FF0000000000000ull;
}

// R^u -= load * fext (no Dirichlet rows replaced)
__global__ void k_sub_load(int n, double load, const double* __restrict__ fext, double* __restrict__ R) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  R[4 * (t / 3) + t % 3] -= load * fext[t];
}

struct FluidState {
  int physics = 0;  // 1 fluid, 2 mesh Laplacian
  double rho = 1.0, mu = 0.0035, dt = 0.125;
  int oseen = 0;    // 1: convective velocity u_old - w (the Oseen step)
  DevBuf<double> dmesh, uold, w;  // [n][3]
};

}  // namespace

// ------------------------------------------------------- library internals
namespace hfsi {

FluidState& fluid_state(hfsi_ctx* c) {
  if (!c->fluid_impl) c->fluid_impl = new FluidState();
  return *reinterpret_cast<FluidState*>(c->fluid_impl);
}

int physics_of(const hfsi_ctx* c) {
  return c->fluid_impl ? reinterpret_cast<const FluidState*>(c->fluid_impl)->physics : 0;
}

void fluid_free(hfsi_ctx* c) {
  delete reinterpret_cast<FluidState*>(c->fluid_impl);
  c->fluid_impl = nullptr;
}

// the element launches of one assembly of a fluid or mesh-Laplacian context
void fluid_elements(hfsi_ctx* c, const double* v, double* R, bool want_K) {
  FluidState& F = fluid_state(c);
  hipStream_t s = c->stream;
  for (size_t q = 0; q + 1 < c->colour_ptr.size(); ++q) {
    const int e0 = c->colour_ptr[q], e1 = c->colour_ptr[q + 1];
    if (F.physics == 1)
      k_fluid_element<<<div_up(e1 - e0, 128), 128, 0, s>>>(
          e0, e1, c->m, c->tets.p, c->X.p, F.dmesh.p, c->V.p, c->slot.p, v, F.uold.p, F.w.p, F.rho, F.mu, F.dt,
          F.oseen, R, c->Kval.p, want_K ? 1 : 0, (unsigned long long*)c->scal.p, c->iscal.p);
    else
      k_laplace_element<<<div_up(e1 - e0, 128), 128, 0, s>>>(e0, e1, c->m, c->tets.p, c->G.p, c->V.p, c->slot.p, v,
                                                             R, c->Kval.p, want_K ? 1 : 0);
    HIP_LAUNCH_CHECK();
  }
}

// the Schur diagonal of the assembled (Dirichlet-eliminated) fluid Jacobian
void fluid_schur(hfsi_ctx* c) {
  k_fluid_schur<<<div_up(c->n, 256), 256, 0, c->stream>>>(c->n, c->nptr.p, c->ncol.p, c->diag_blk.p, c->Kval.p,
                                                           c->schur.p);
  HIP_LAUNCH_CHECK();
}

// raw fluid residual at state v and load factor `load` (element terms minus
// the inlet load, no Dirichlet rows replaced) into R [4n]
void fluid_residual_raw(hfsi_ctx* c, const double* v, double load, double* R) {
  hipStream_t s = c->stream;
  const int n = c->n;
  c->iscal.ensure(16);
  c->scal.ensure(16);
  HIP_CHECK(hipMemsetAsync(R, 0, sizeof(double) * 4 * (size_t)n, s));
  k_flags<<<1, 1, 0, s>>>(c->iscal.p, (unsigned long long*)c->scal.p);
  HIP_LAUNCH_CHECK();
  fluid_elements(c, v, R, false);
  k_sub_load<<<div_up(3 * n, 256), 256, 0, s>>>(n, load, c->fext.p, R);
  HIP_LAUNCH_CHECK();
  int inv = 0;
  HIP_CHECK(hipMemcpyAsync(&inv, c->iscal.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (inv != INT32_MAX) fail(HFSI_E_INVERTED, "element " + std::to_string(c->perm[inv]) + " of the moved mesh is inverted");
}

}  // namespace hfsi

namespace {

void require_fluid(hfsi_ctx* c, const char* what) {
  if (physics_of(c) != 1) fail(HFSI_E_ORDER, std::string(what) + ": the context is not a fluid (hfsi_set_fluid)");
}

void upload_field(hfsi_ctx* c, DevBuf<double>& dst, const double* src) {
  if (src) HIP_CHECK(hipMemcpyAsync(dst.p, src, sizeof(double) * 3 * (size_t)c->n, hipMemcpyDeviceToDevice, c->stream));
}

}  // namespace

extern "C" hfsi_status hfsi_set_fluid(hfsi_ctx* c, double rho, double mu, double dt, int32_t oseen) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 1, "set_fluid");
  if (!(rho > 0.0) || !(mu >= 0.0) || !(dt > 0.0) || oseen < 0 || oseen > 1)
    fail(HFSI_E_ARG, "set_fluid: need rho > 0, mu >= 0, dt > 0, oseen 0 or 1");
  FluidState& F = fluid_state(c);
  F.physics = 1;
  F.rho = rho;
  F.mu = mu;
  F.dt = dt;
  F.oseen = oseen;
  F.dmesh.zero(3 * (size_t)c->n, c->stream);
  F.uold.zero(3 * (size_t)c->n, c->stream);
  F.w.zero(3 * (size_t)c->n, c->stream);
  c->cm = 0.0;
  c->H.reusable = false;
  vanka_invalidate(c);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_set_fluid_fields(hfsi_ctx* c, const double* dmesh, const double* u_old, const double* w) {
  HFSI_ABI_BEGIN(c)
  require_fluid(c, "set_fluid_fields");
  FluidState& F = fluid_state(c);
  upload_field(c, F.dmesh, dmesh);
  upload_field(c, F.uold, u_old);
  upload_field(c, F.w, w);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_set_mesh_laplace(hfsi_ctx* c) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 2, "set_mesh_laplace");
  FluidState& F = fluid_state(c);
  F.physics = 2;
  c->cm = 0.0;
  c->schur.ensure(c->n);
  k_fill<<<div_up(c->n, 256), 256, 0, c->stream>>>(c->n, 1.0, c->schur.p);
  HIP_LAUNCH_CHECK();
  vanka_invalidate(c);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_fluid_interface_force(hfsi_ctx* c, const double* v, double load, int32_t count,
                                                  const int32_t* nodes, double* f) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 3, "fluid_interface_force");
  require_fluid(c, "fluid_interface_force");
  if (!v || !f || count < 0 || (count > 0 && !nodes)) fail(HFSI_E_ARG, "fluid_interface_force: bad arguments");
  std::vector<int> idx(nodes, nodes + count);
  for (int k : idx)
    if (k < 0 || k >= c->n) fail(HFSI_E_ARG, "fluid_interface_force: node out of range");
  hipStream_t s = c->stream;
  DevBuf<int> di;
  DevBuf<double> R;
  di.upload(idx.data(), idx.size(), s);
  R.ensure(4 * (size_t)c->n);
  fluid_residual_raw(c, v, load, R.p);
  if (count) {
    k_force<<<div_up(3 * count, 256), 256, 0, s>>>(count, di.p, R.p, f);
    HIP_LAUNCH_CHECK();
  }
  HIP_CHECK(hipStreamSynchronize(s));
  HFSI_ABI_END(c)
}

// ------------------------------------------------------------------ FSI step

namespace {

struct FsiWork {
  DevBuf<int> fidx, sidx;
  DevBuf<double> dG, r, rp, f, dots, vm, dprev, vs_prev, Rf;
};

void check_fsi_params(const hfsi_fsi_params* p) {
  if (!p || p->struct_size != sizeof(hfsi_fsi_params)) fail(HFSI_E_ARG, "fsi params: struct_size mismatch");
  if (!(p->omega0 > 0.0) || !(p->eps > 0.0) || p->max_dn < 1 || p->max_dn > 128 || !(p->eps2 > 0.0) ||
      p->adaptive < 0 || p->adaptive > 1)
    fail(HFSI_E_ARG, "fsi params: need omega0 > 0, eps > 0, 1 <= max_dn <= 128, eps2 > 0, adaptive 0 or 1");
}

}  // namespace

extern "C" hfsi_status hfsi_fsi_time_step(hfsi_ctx* fl, hfsi_ctx* me, hfsi_ctx* so, int32_t n_iface,
                                          const int32_t* iface_f, const int32_t* iface_s, double* vf, double* df,
                                          double* vs, double* vel, double* acc, double inlet_load,
                                          const hfsi_fsi_params* prm, hfsi_fsi_info* info) {
  HFSI_ABI_BEGIN(fl)
  if (!me || !so) fail(HFSI_E_ARG, "fsi_time_step: null context");
  if (me->device != fl->device || so->device != fl->device) fail(HFSI_E_ARG, "fsi_time_step: contexts on different devices");
  require_stage(fl, 3, "fsi_time_step (fluid)");
  require_stage(me, 3, "fsi_time_step (mesh)");
  require_stage(so, 3, "fsi_time_step (structure)");
  require_fluid(fl, "fsi_time_step");
  if (physics_of(me) != 2) fail(HFSI_E_ORDER, "fsi_time_step: the mesh context is not a Laplacian (hfsi_set_mesh_laplace)");
  if (physics_of(so) != 0 || !(so->cm > 0.0)) fail(HFSI_E_ORDER, "fsi_time_step: the structure needs Newmark inertia");
  if (me->n != fl->n) fail(HFSI_E_ARG, "fsi_time_step: fluid and mesh contexts on different meshes");
  check_fsi_params(prm);
  if (info && info->struct_size != sizeof(hfsi_fsi_info)) fail(HFSI_E_ARG, "fsi info: struct_size mismatch");
  if (n_iface < 1 || !iface_f || !iface_s || !vf || !df || !vs || !vel || !acc)
    fail(HFSI_E_ARG, "fsi_time_step: bad arguments");
  for (int k = 0; k < n_iface; ++k)
    if (iface_f[k] < 0 || iface_f[k] >= fl->n || iface_s[k] < 0 || iface_s[k] >= so->n)
      fail(HFSI_E_ARG, "fsi_time_step: interface node out of range");
  auto t0 = std::chrono::steady_clock::now();
  // every context queues on its own stream; the step runs on the fluid's and
  // waits for the others' at each hand-over by synchronising them
  hipStream_t s = fl->stream;
  FluidState& F = fluid_state(fl);
  const int nf = fl->n, ns = so->n, len = 3 * n_iface;
  const double dt = F.dt;
  FsiWork W;
  W.fidx.upload(iface_f, n_iface, s);
  W.sidx.upload(iface_s, n_iface, s);
  W.dG.ensure(len);
  W.r.ensure(len);
  W.rp.ensure(len);
  W.f.ensure(len);
  W.dots.ensure(4);
  W.vm.zero(4 * (size_t)nf, s);
  W.dprev.ensure(3 * (size_t)nf);
  W.vs_prev.ensure(4 * (size_t)ns);
  W.Rf.ensure(4 * (size_t)nf);
  HIP_CHECK(hipMemcpyAsync(W.dprev.p, df, sizeof(double) * 3 * nf, hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipMemcpyAsync(W.vs_prev.p, vs, sizeof(double) * 4 * ns, hipMemcpyDeviceToDevice, s));
  k_u_of<<<div_up(3 * nf, 256), 256, 0, s>>>(nf, vf, F.uold.p);
  k_predict<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.sidx.p, vs, vel, dt, W.dG.p);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipStreamSynchronize(s));
  hfsi_status st = hfsi_newmark_history(so, W.vs_prev.p, vel, acc);
  if (st < 0) {
    fl->err = std::string("fsi_time_step: structure: ") + so->err;
    return st;
  }
  HIP_CHECK(hipStreamSynchronize(so->stream));
  hfsi_newton_solve_params pf{}, ps{};
  pf.struct_size = ps.struct_size = sizeof(hfsi_newton_solve_params);
  pf.step = prm->fluid_step;
  ps.step = prm->solid_step;
  pf.eps2 = ps.eps2 = prm->eps2;
  pf.max_newton = ps.max_newton = 25;
  pf.eps1_max = ps.eps1_max = 1e-2;
  pf.eps1_min = ps.eps1_min = 1e-12;
  pf.ref_norm = ps.ref_norm = 0.0;
  pf.adaptive = ps.adaptive = prm->adaptive;
  hfsi_newton_params pm = prm->mesh_step;
  int k = 0, fl_its = 0, so_its = 0, kry = 0;
  bool done = false;
  double omega = prm->omega0;
  auto sub_fail = [&](hfsi_ctx* who, const char* name, hfsi_status code) {
    fl->err = std::string("fsi_time_step: ") + name + " (DN iteration " + std::to_string(k) +
              "): " + (who->err.empty() ? "not converged" : who->err);
    if (info) {  // the iterations so far (residual and omega of the earlier ones)
      info->dn_iterations = k;
      info->fluid_newton = fl_its;
      info->solid_newton = so_its;
      info->krylov = kry;
      info->converged = 0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return code < 0 ? code : HFSI_E_BREAKDOWN;
  };
  for (k = 1; k <= prm->max_dn; ++k) {
    // 1. harmonic extension of dG, mesh displacement and velocity
    k_scatter_u<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.fidx.p, W.dG.p, W.vm.p);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(s));
    hfsi_newton_info mi{sizeof(hfsi_newton_info)};
    st = hfsi_newton_step(me, W.vm.p, 0.0, &pm, &mi);
    if (st != HFSI_OK) return sub_fail(me, "mesh extension", st);
    kry += mi.krylov_iterations;
    HIP_CHECK(hipStreamSynchronize(me->stream));
    k_mesh_motion<<<div_up(3 * nf, 256), 256, 0, s>>>(nf, W.vm.p, W.dprev.p, dt, F.dmesh.p, F.w.p);
    // 2. the fluid, with the mesh velocity on the interface
    k_set_iface_velocity<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.fidx.p, F.w.p, vf);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(s));
    hfsi_newton_solve_info fi{sizeof(hfsi_newton_solve_info)};
    st = hfsi_newton_solve(fl, vf, inlet_load, &pf, &fi);
    fl_its += fi.newton_iterations;
    kry += fi.krylov_iterations;
    if (st != HFSI_OK) return sub_fail(fl, "fluid", st);
    if (pf.ref_norm == 0.0) pf.ref_norm = fi.dv_mass_norm[0] > 0.0 ? fi.dv_mass_norm[0] : 0.0;
    // 3. the fluid's force on the wall as the structure's load, then the structure
    fluid_residual_raw(fl, vf, inlet_load, W.Rf.p);
    k_force<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.fidx.p, W.Rf.p, W.f.p);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipMemsetAsync(so->fext.p, 0, sizeof(double) * 3 * ns, s));
    k_load_scatter<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.sidx.p, W.f.p, so->fext.p);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipStreamSynchronize(s));
    hfsi_newton_solve_info si{sizeof(hfsi_newton_solve_info)};
    st = hfsi_newton_solve(so, vs, 1.0, &ps, &si);
    so_its += si.newton_iterations;
    kry += si.krylov_iterations;
    if (st != HFSI_OK) return sub_fail(so, "structure", st);
    if (ps.ref_norm == 0.0) ps.ref_norm = si.dv_mass_norm[0] > 0.0 ? si.dv_mass_norm[0] : 0.0;
    HIP_CHECK(hipStreamSynchronize(so->stream));
    // interface residual, stopping rule, Aitken factor, relaxation
    k_iface_residual<<<div_up(len, 256), 256, 0, s>>>(n_iface, W.sidx.p, vs, W.dG.p, W.r.p);
    k_iface_dots<<<1, 256, 0, s>>>(len, W.r.p, k > 1 ? W.rp.p : nullptr, W.dots.p);
    HIP_LAUNCH_CHECK();
    double dots[3];
    HIP_CHECK(hipMemcpyAsync(dots, W.dots.p, sizeof(dots), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    const double norm = std::sqrt(dots[0]) / std::sqrt((double)n_iface);
    if (info && k <= 128) info->residual[k - 1] = norm;
    if (!std::isfinite(norm)) fail(HFSI_E_NAN, "fsi_time_step: non-finite interface residual");
    if (norm < prm->eps) {
      done = true;
      break;
    }
    if (k > 1) {
      if (!(dots[2] > 0.0)) fail(HFSI_E_BREAKDOWN, "fsi_time_step: equal interface residuals (Aitken undefined)");
      omega = -omega * dots[1] / dots[2];
    }
    if (info && k <= 128) info->omega[k - 1] = omega;
    k_relax<<<div_up(len, 256), 256, 0, s>>>(len, omega, W.r.p, W.dG.p, W.rp.p);
    HIP_LAUNCH_CHECK();
  }
  if (info) {
    info->dn_iterations = std::min(k, prm->max_dn);
    info->fluid_newton = fl_its;
    info->solid_newton = so_its;
    info->krylov = kry;
    info->converged = done ? 1 : 0;
  }
  if (!done) {
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fl->err = "fsi_time_step: the DN iteration did not converge";
    return HFSI_NOT_CONVERGED;
  }
  // end of step: Newmark update of the structure, the new mesh displacement
  st = hfsi_newmark_update(so, vs, W.vs_prev.p, vel, acc);
  if (st < 0) return sub_fail(so, "structure update", st);
  HIP_CHECK(hipStreamSynchronize(so->stream));
  HIP_CHECK(hipMemcpyAsync(df, F.dmesh.p, sizeof(double) * 3 * nf, hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  HFSI_ABI_END(fl)
}
