// Element residual and consistent tangent of the stabilised P1-P1 solid,
// atomic-free global assembly by element colours, Dirichlet elimination and
// extraction of the displacement block A.
//
// Per tetrahedron (one centroid point; F, J, S' are constant on a P1 tet):
//   R^u_a = V (F S' G_a - pbar J g_a),                      g_a = F^{-T} G_a
//   R^p_a = -V/4 (J-1) - 1/kappa sum_b M_ab p_b - tau V J g_a . ghat,
//           ghat = F^{-T} grad p,  M_ab = V (1+delta_ab)/20,  tau = h^2/(4 mu^l)
// (weak residuals of the structure with the PSPG term of eq. stelas), with
// the Newmark-beta inertia when it is on (cm = rho_s/(beta dt^2), r_b the
// nodal history field r_s, m = V/4 sum_b (r_b - cm d_b) / V the element mean
// of r_s - cm d):
//   R^u_a += sum_b M_ab (cm d_b - r_b),   R^p_a += tau V g_a . m,
//   A_ab  += cm M_ab I,                   B2_ab += tau V (-cm/4 - g_b . m) g_a^T,
// and the exact derivative K = [A B1^T; B2 -C] (eq. globsys):
//   A_ab  = V [ (G_a.S'G_b) I + B_a^T D B_b ] - pbar V J (g_a g_b^T - g_b g_a^T)
//   B1^T_ab = -V/4 J g_a
//   B2_ab = -V/4 J g_b^T - tau V J [ (g_a.ghat) g_b^T - (g_b.ghat) g_a^T - (g_a.g_b) ghat^T ]
//   C_ab  = M_ab / kappa + tau V J g_a.g_b
// with D the 6x6 Voigt matrix of C' = 2 dS'/dC and B_a the Green-Lagrange
// strain variation of node a.  S' and C' follow eq. mmrpkt/mmrpktmix
// (Mooney-Rivlin) and eq. arpkt/arpktmix (artery; the fibre stress carries
// the 2 k1 factor of S = 2 dPsi/dC, fibres act only while J_i > 1).
#include <cmath>
#include <mutex>
#include <string>

#include "common.hpp"

using namespace hfsi;

namespace {

// Voigt pairs (11, 22, 33, 12, 23, 13)
__device__ __constant__ int VI[6] = {0, 1, 2, 0, 1, 0};
__device__ __constant__ int VJ[6] = {0, 1, 2, 1, 2, 2};

struct Sym {  // symmetric 3x3 in Voigt order
  double v[6];
};

__device__ __forceinline__ double sget(const double (&A)[3][3], int p) { return A[VI[p]][VJ[p]]; }

// (A (.) A)_{IJKL} = 1/2 (A_IK A_JL + A_IL A_JK) for Voigt pairs p=(I,J), q=(K,L)
__device__ __forceinline__ double odot(const double (&A)[3][3], int p, int q) {
  const int I = VI[p], J = VJ[p], K = VI[q], L = VJ[q];
  return 0.5 * (A[I][K] * A[J][L] + A[I][L] * A[J][K]);
}

__device__ __forceinline__ double symid(int p, int q) {
  if (p != q) return 0.0;
  return p < 3 ? 1.0 : 0.5;
}

// Stress S' (3x3) and Voigt tangent D of one element.
__device__ void material(const double (&C)[3][3], const double (&Ci)[3][3], double I3, const double* mt,
                         const double* a1, const double* a2, double (&S)[3][3], double (&D)[6][6]) {
  const int model = (int)mt[0];
  const double c10 = mt[1], c01 = mt[2], k1 = mt[4], k2 = mt[5];
  const double I1 = C[0][0] + C[1][1] + C[2][2];
  double CC = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) CC += C[i][j] * C[i][j];
  const double I2 = 0.5 * (I1 * I1 - CC);
  const double r13 = 1.0 / cbrt(I3);
  const double r23 = r13 * r13;
  double Cv[6], Civ[6], Bv[6], Iv[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    Cv[p] = sget(C, p);
    Civ[p] = sget(Ci, p);
    Iv[p] = p < 3 ? 1.0 : 0.0;
    Bv[p] = I1 * Iv[p] - Cv[p];
  }
  // S' : J1 and J2 parts
  double Sv[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    Sv[p] = c10 * r13 * (Iv[p] - (I1 / 3.0) * Civ[p]);
    if (model == 0) Sv[p] += c01 * r23 * (Bv[p] - (2.0 * I2 / 3.0) * Civ[p]);
  }
  const double t1 = 2.0 * c10 * r13;
  const double t2 = 2.0 * c01 * r23;
#pragma unroll
  for (int p = 0; p < 6; ++p)
#pragma unroll
    for (int q = p; q < 6; ++q) {
      const double cc = odot(Ci, p, q);
      double d = t1 * (-(Iv[p] * Civ[q] + Civ[p] * Iv[q]) / 3.0 + (I1 / 9.0) * Civ[p] * Civ[q] + (I1 / 3.0) * cc);
      if (model == 0)
        d += t2 * (Iv[p] * Iv[q] - symid(p, q) - (2.0 / 3.0) * (Bv[p] * Civ[q] + Civ[p] * Bv[q]) +
                   (4.0 * I2 / 9.0) * Civ[p] * Civ[q] + (2.0 * I2 / 3.0) * cc);
      D[p][q] = d;
    }
  if (model == 1) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const double* a = f == 0 ? a1 : a2;
      double Av[6];
#pragma unroll
      for (int p = 0; p < 6; ++p) Av[p] = a[VI[p]] * a[VJ[p]];
      double I4 = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I4 += a[i] * a[j] * C[i][j];
      const double Ji = r13 * I4;
      if (Ji > 1.0) {
        const double x = Ji - 1.0;
        const double ex = exp(k2 * x * x);
        const double d1 = k1 * x * ex;                         // psi'
        const double d2 = k1 * ex * (1.0 + 2.0 * k2 * x * x);  // psi''
        double Dv[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) {
          Dv[p] = r13 * (Av[p] - (I4 / 3.0) * Civ[p]);
          Sv[p] += 2.0 * d1 * Dv[p];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
          for (int q = p; q < 6; ++q) {
            const double dD = r13 * (-(Av[p] * Civ[q] + Civ[p] * Av[q]) / 3.0 + (I4 / 9.0) * Civ[p] * Civ[q] +
                                     (I4 / 3.0) * odot(Ci, p, q));
            D[p][q] += 4.0 * (d2 * Dv[p] * Dv[q] + d1 * dD);
          }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 6; ++p)
#pragma unroll
    for (int q = 0; q < p; ++q) D[p][q] = D[q][p];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    S[VI[p]][VJ[p]] = Sv[p];
    S[VJ[p]][VI[p]] = Sv[p];
  }
}

// strain variation of node a, component i (engineering Voigt)
__device__ __forceinline__ void bvec(const double (&F)[3][3], const double* g, int i, double (&b)[6]) {
  b[0] = F[i][0] * g[0];
  b[1] = F[i][1] * g[1];
  b[2] = F[i][2] * g[2];
  b[3] = F[i][0] * g[1] + F[i][1] * g[0];
  b[4] = F[i][1] * g[2] + F[i][2] * g[1];
  b[5] = F[i][0] * g[2] + F[i][2] * g[0];
}

__global__ void __launch_bounds__(128)
k_element(int e0, int e1, int m, const int* __restrict__ T, const int* __restrict__ mat,
          const double* __restrict__ mtab, const double* __restrict__ Gs, const double* __restrict__ Vs,
          const double* __restrict__ Hs, const double* __restrict__ fib, const int* __restrict__ slot,
          const double* __restrict__ v, double* __restrict__ R, double* __restrict__ Kval, int want_K,
          unsigned long long* __restrict__ minJ, int* __restrict__ inverted, double cm,
          const double* __restrict__ rs) {
  const int e = e0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  int nd[4];
  double G[4][3], u[4][3], p[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nd[a] = T[a * m + e];
#pragma unroll
    for (int J = 0; J < 3; ++J) G[a][J] = Gs[(a * 3 + J) * m + e];
    const double2 v01 = *reinterpret_cast<const double2*>(v + 4 * nd[a]);
    const double2 v23 = *reinterpret_cast<const double2*>(v + 4 * nd[a] + 2);
    u[a][0] = v01.x;
    u[a][1] = v01.y;
    u[a][2] = v23.x;
    p[a] = v23.y;
  }
  const double V = Vs[e];
  const double* mt = mtab + 8 * mat[e];
  const double kappa = mt[3];
  const double tau = Hs[e] * Hs[e] / (4.0 * mt[6]);
  double a1[3] = {0, 0, 0}, a2[3] = {0, 0, 0};
  if ((int)mt[0] == 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      a1[i] = fib[i * m + e];
      a2[i] = fib[(3 + i) * m + e];
    }
  }
  // kinematics
  double F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      F[i][J] = (i == J ? 1.0 : 0.0) + u[0][i] * G[0][J] + u[1][i] * G[1][J] + u[2][i] * G[2][J] + u[3][i] * G[3][J];
  const double c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  const double c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  const double c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  const double Jd = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
  if (!(Jd > 0.0)) {
    atomicMin(inverted, e);
    return;
  }
  // smallest J: the atomic only when J is below the value already recorded
  // (many atomics on one address serialise)
  const unsigned long long jbits = (unsigned long long)__double_as_longlong(Jd);
  if (jbits < __hip_atomic_load(minJ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(minJ, jbits);
  const double iJ = 1.0 / Jd;
  double Fi[3][3];
  Fi[0][0] = c00 * iJ;
  Fi[1][0] = c01 * iJ;
  Fi[2][0] = c02 * iJ;
  Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * iJ;
  Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * iJ;
  Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * iJ;
  Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * iJ;
  Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * iJ;
  Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * iJ;
  double C[3][3], Ci[3][3];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      C[I][J] = F[0][I] * F[0][J] + F[1][I] * F[1][J] + F[2][I] * F[2][J];
      Ci[I][J] = Fi[I][0] * Fi[J][0] + Fi[I][1] * Fi[J][1] + Fi[I][2] * Fi[J][2];
    }
  double S[3][3], D[6][6];
  material(C, Ci, Jd * Jd, mt, a1, a2, S, D);

  // spatial gradients g_a = F^{-T} G_a, pressure quantities
  double g[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) g[a][i] = Fi[0][i] * G[a][0] + Fi[1][i] * G[a][1] + Fi[2][i] * G[a][2];
  const double pbar = 0.25 * (p[0] + p[1] + p[2] + p[3]);
  double gp[3], gh[3];
#pragma unroll
  for (int J = 0; J < 3; ++J) gp[J] = p[0] * G[0][J] + p[1] * G[1][J] + p[2] * G[2][J] + p[3] * G[3][J];
#pragma unroll
  for (int i = 0; i < 3; ++i) gh[i] = Fi[0][i] * gp[0] + Fi[1][i] * gp[1] + Fi[2][i] * gp[2];
  double gdot[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) gdot[a] = g[a][0] * gh[0] + g[a][1] * gh[1] + g[a][2] * gh[2];
  // inertia: ru_b = cm d_b - r_b, mv = mean of r_s - cm d, gm_a = g_a . mv
  const bool dyn = rs != nullptr;
  double ru[4][3], gm[4] = {0.0, 0.0, 0.0, 0.0};
  if (dyn) {
    double mv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        ru[a][i] = cm * u[a][i] - rs[3 * nd[a] + i];
        mv[i] -= 0.25 * ru[a][i];
      }
#pragma unroll
    for (int a = 0; a < 4; ++a) gm[a] = g[a][0] * mv[0] + g[a][1] * mv[1] + g[a][2] * mv[2];
  }
  const double VJ_ = V * Jd;
  const double tVJ = tau * V * Jd;
  double FS[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) FS[i][J] = F[i][0] * S[0][J] + F[i][1] * S[1][J] + F[i][2] * S[2][J];

  // residual
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double* Ra = R + 4 * nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      Ra[i] += V * (FS[i][0] * G[a][0] + FS[i][1] * G[a][1] + FS[i][2] * G[a][2]) - pbar * VJ_ * g[a][i];
    double Mp = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) Mp += (a == b ? 2.0 : 1.0) * p[b];
    Mp *= V / 20.0;
    Ra[3] += -0.25 * V * (Jd - 1.0) - Mp / kappa - tVJ * gdot[a];
    if (dyn) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double Mr = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) Mr += (a == b ? 2.0 : 1.0) * ru[b][i];
        Ra[i] += V / 20.0 * Mr;
      }
      Ra[3] += tau * V * gm[a];
    }
  }
  if (!want_K) return;

  // tangent, block by block
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    double DB[3][6];  // D B_a (rows = component i)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double b[6];
      bvec(F, G[a], i, b);
#pragma unroll
      for (int q = 0; q < 6; ++q)
        DB[i][q] = D[q][0] * b[0] + D[q][1] * b[1] + D[q][2] * b[2] + D[q][3] * b[3] + D[q][4] * b[4] + D[q][5] * b[5];
    }
    double SGa[3];
#pragma unroll
    for (int J = 0; J < 3; ++J) SGa[J] = S[J][0] * G[a][0] + S[J][1] * G[a][1] + S[J][2] * G[a][2];
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      double blk[16];
      const double geo = V * (SGa[0] * G[b][0] + SGa[1] * G[b][1] + SGa[2] * G[b][2]);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double bb[6];
        bvec(F, G[b], k, bb);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double mm = DB[i][0] * bb[0] + DB[i][1] * bb[1] + DB[i][2] * bb[2] + DB[i][3] * bb[3] + DB[i][4] * bb[4] +
                      DB[i][5] * bb[5];
          double val = V * mm - pbar * VJ_ * (g[a][i] * g[b][k] - g[b][i] * g[a][k]);
          if (i == k) val += geo;
          if (dyn && i == k) val += cm * (a == b ? 2.0 : 1.0) * V / 20.0;
          blk[i * 4 + k] = val;
        }
      }
      const double gab = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) blk[i * 4 + 3] = -0.25 * VJ_ * g[a][i];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        blk[12 + k] = -0.25 * VJ_ * g[b][k] - tVJ * (gdot[a] * g[b][k] - gdot[b] * g[a][k] - gab * gh[k]);
      if (dyn)
#pragma unroll
        for (int k = 0; k < 3; ++k) blk[12 + k] += tau * V * (-0.25 * cm - gm[b]) * g[a][k];
      blk[15] = -((a == b ? 2.0 : 1.0) * V / 20.0 / kappa + tVJ * gab);
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

__global__ void k_init_flags(int* inverted, unsigned long long* minJ) {
  *inverted = INT32_MAX;
  *minJ = 0x7FF0000000000000ull;  // +inf
}

// external load and Dirichlet rows of the residual
__global__ void k_residual_bc(int n, double load, const double* __restrict__ fext, const uint8_t* __restrict__ dir,
                              double* __restrict__ R) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double r = R[4 * i + c];
    if (c < 3) r -= load * fext[3 * i + c];
    if (dir[4 * i + c]) r = 0.0;
    R[4 * i + c] = r;
  }
}

// Dirichlet elimination in the block matrix: zero rows/columns of fixed dofs,
// unit diagonal.
__global__ void k_dirichlet_K(int nb, const int* __restrict__ brow, const int* __restrict__ bcol,
                              const uint8_t* __restrict__ dir, double* __restrict__ Kval) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 16 * nb) return;
  int q = t >> 4, r = (t >> 2) & 3, c = t & 3;
  int i = brow[q], j = bcol[q];
  if (dir[4 * i + r] || dir[4 * j + c]) Kval[t] = (i == j && r == c) ? 1.0 : 0.0;
}

// A pattern: row 3i+r keeps column 3j+c of block (i,j) unless the row or the
// column dof is fixed (the diagonal is always kept).
__global__ void k_a_count(int n, const int* __restrict__ nptr, const int* __restrict__ ncol,
                          const uint8_t* __restrict__ dir, int* __restrict__ cnt) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  int i = t / 3, r = t % 3;
  if (dir[4 * i + r]) { cnt[t] = 1; return; }
  int k = 0;
  for (int q = nptr[i]; q < nptr[i + 1]; ++q) {
    int j = ncol[q];
    for (int c = 0; c < 3; ++c) k += dir[4 * j + c] ? 0 : 1;
  }
  cnt[t] = k;
}

__global__ void k_a_fill(int n, const int* __restrict__ nptr, const int* __restrict__ ncol,
                         const uint8_t* __restrict__ dir, const int* __restrict__ aptr, int* __restrict__ acol,
                         int* __restrict__ src) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  int i = t / 3, r = t % 3;
  int o = aptr[t];
  for (int q = nptr[i]; q < nptr[i + 1]; ++q) {
    int j = ncol[q];
    for (int c = 0; c < 3; ++c) {
      bool keep = dir[4 * i + r] ? (j == i && c == r) : !dir[4 * j + c];
      if (keep) {
        acol[o] = 3 * j + c;
        src[o] = 16 * q + 4 * r + c;
        ++o;
      }
    }
  }
}

__global__ void k_gather(int nnz, const int* __restrict__ src, const double* __restrict__ Kval,
                         double* __restrict__ val) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) val[t] = Kval[src[t]];
}

// compact copy of B2: the pressure row, displacement columns, of every block
__global__ void k_extract_b2(int nb, const double* __restrict__ Kval, double* __restrict__ b2) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * nb) return;
  const int q = t / 3, c = t - 3 * q;
  b2[t] = Kval[16 * (size_t)q + 12 + c];
}

// ||dv||_M from the partials of k_massnorm: one block of kNoallocParts
// threads folds them in the order k_sum_partial + k_sum_final fold the same
// values (slot t to thread t, then the halving tree) and writes the root
__global__ void __launch_bounds__(256) k_massnorm_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[256];
  sh[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0] > 0.0 ? sh[0] : 0.0);
}

// mass norm partials: sum over blocks (i,j) of M_ij sum_c dv_ic dv_jc
__global__ void k_massnorm(int nb, const int* __restrict__ brow, const int* __restrict__ bcol,
                           const double* __restrict__ M, const double* __restrict__ dv, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < nb; q += gridDim.x * 256) {
    const int i = brow[q], j = bcol[q];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += dv[4 * i + c] * dv[4 * j + c];
    acc += M[q] * s;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

}  // namespace

namespace hfsi {

void build_a_pattern(hfsi_ctx* c) {
  const int n = c->n;
  hipStream_t s = c->stream;
  DevBuf<int> cnt;
  cnt.ensure(3 * (size_t)n + 1);
  HIP_CHECK(hipMemsetAsync(cnt.p + 3 * n, 0, sizeof(int), s));
  k_a_count<<<div_up(3 * n, 256), 256, 0, s>>>(n, c->nptr.p, c->ncol.p, c->dir.p, cnt.p);
  HIP_LAUNCH_CHECK();
  c->A.ptr.ensure(3 * (size_t)n + 1);
  int64_t nnz = exclusive_scan(cnt.p, c->A.ptr.p, 3 * n + 1, s);
  if (nnz > INT32_MAX) fail(HFSI_E_ARG, "A exceeds int32 indexing");
  c->A.rows = c->A.cols = 3 * n;
  c->A.nnz = nnz;
  c->A.col.ensure(nnz);
  c->A.val.ensure(nnz);
  c->a_src.ensure(nnz);
  k_a_fill<<<div_up(3 * n, 256), 256, 0, s>>>(n, c->nptr.p, c->ncol.p, c->dir.p, c->A.ptr.p, c->A.col.p, c->a_src.p);
  HIP_LAUNCH_CHECK();
}

void assemble(hfsi_ctx* c, const double* v, double load, double* R, hfsi_assembly_info* info) {
  hipStream_t s = c->stream;
  const int n = c->n, m = c->m;
  c->iscal.ensure(16);
  c->scal.ensure(16);
  HIP_CHECK(hipEventRecord(c->ev0, s));
  HIP_CHECK(hipMemsetAsync(R, 0, sizeof(double) * 4 * (size_t)n, s));
  HIP_CHECK(hipMemsetAsync(c->Kval.p, 0, sizeof(double) * 16 * (size_t)c->nb, s));
  k_init_flags<<<1, 1, 0, s>>>(c->iscal.p, (unsigned long long*)c->scal.p);
  HIP_LAUNCH_CHECK();
  const int physics = physics_of(c);
  if (physics != 0) {
    fluid_elements(c, v, R, true);
  } else {
    for (size_t q = 0; q + 1 < c->colour_ptr.size(); ++q) {
      int e0 = c->colour_ptr[q], e1 = c->colour_ptr[q + 1];
      k_element<<<div_up(e1 - e0, 128), 128, 0, s>>>(e0, e1, m, c->tets.p, c->mat.p, c->mtab.p, c->G.p, c->V.p,
                                                     c->h.p, c->has_fib ? c->fib.p : nullptr, c->slot.p, v, R,
                                                     c->Kval.p, 1, (unsigned long long*)c->scal.p, c->iscal.p, c->cm,
                                                     c->cm > 0.0 ? c->rs.p : nullptr);
      HIP_LAUNCH_CHECK();
    }
  }
  k_residual_bc<<<div_up(n, 256), 256, 0, s>>>(n, load, c->fext.p, c->dir.p, R);
  HIP_LAUNCH_CHECK();
  k_dirichlet_K<<<div_up(16 * (long)c->nb, 256), 256, 0, s>>>(c->nb, c->brow.p, c->ncol.p, c->dir.p, c->Kval.p);
  HIP_LAUNCH_CHECK();
  if (physics == 1) fluid_schur(c);
  k_gather<<<div_up(c->A.nnz, 256), 256, 0, s>>>((int)c->A.nnz, c->a_src.p, c->Kval.p, c->A.val.p);
  HIP_LAUNCH_CHECK();
  c->b2.ensure(3 * (size_t)c->nb);
  k_extract_b2<<<div_up(3L * c->nb, 256), 256, 0, s>>>(c->nb, c->Kval.p, c->b2.p);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipEventRecord(c->ev1, s));
  int inv = 0;
  double minJ = 0;
  HIP_CHECK(hipMemcpyAsync(&inv, c->iscal.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&minJ, c->scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (inv != INT32_MAX)
    fail(HFSI_E_INVERTED, "element " + std::to_string(c->perm[inv]) + " has J <= 0");
  if (info) {
    info->seconds = elapsed_ms(c) * 1e-3;
    info->n_colours = (int)c->colour_ptr.size() - 1;
    info->min_J = minJ;
  }
}

// Per element: gradients (96 B), volume and size (16 B), connectivity (16 B),
// material id (4 B), fibres (48 B, anisotropic meshes); per node the state
// (32 B) and, with inertia, the history field (24 B); the tangent values (8 B per scalar entry) and the residual (8 B per
// dof) written once.
double assembly_bytes(hfsi_ctx* c) {
  const double per_elem = 96.0 + 16.0 + 16.0 + 4.0 + (c->has_fib ? 48.0 : 0.0);
  return c->m * per_elem + c->n * (32.0 + (c->cm > 0.0 ? 24.0 : 0.0)) + 16.0 * c->nb * 8.0 + 4.0 * c->n * 8.0;
}

// The colour launches of one assembly at the zero state (timing only).
void assemble_kernels_only(hfsi_ctx* c) {
  hipStream_t s = c->stream;
  const long N = 4L * c->n;
  c->kdv.ensure(N);
  c->ktmp.ensure(N);
  c->iscal.ensure(16);
  c->scal.ensure(16);
  HIP_CHECK(hipMemsetAsync(c->kdv.p, 0, sizeof(double) * N, s));
  HIP_CHECK(hipMemsetAsync(c->ktmp.p, 0, sizeof(double) * N, s));
  HIP_CHECK(hipMemsetAsync(c->Kval.p, 0, sizeof(double) * 16 * (size_t)c->nb, s));
  for (size_t q = 0; q + 1 < c->colour_ptr.size(); ++q) {
    int e0 = c->colour_ptr[q], e1 = c->colour_ptr[q + 1];
    k_element<<<div_up(e1 - e0, 128), 128, 0, s>>>(e0, e1, c->m, c->tets.p, c->mat.p, c->mtab.p, c->G.p, c->V.p,
                                                   c->h.p, c->has_fib ? c->fib.p : nullptr, c->slot.p, c->kdv.p,
                                                   c->ktmp.p, c->Kval.p, 1, (unsigned long long*)c->scal.p,
                                                   c->iscal.p, c->cm, c->cm > 0.0 ? c->rs.p : nullptr);
    HIP_LAUNCH_CHECK();
  }
}

// ------------------------------------------- allocation-free mass norm
// The block partial sums of k_massnorm for hfsi_mass_norm_noalloc live in a
// file-scope device array: one copy per GPU, held until the process ends,
// shared by every call on that GPU (calls that overlap on one GPU race on
// it).  k_massnorm writes every slot before the final kernel reads it, so
// nothing needs clearing between calls.  Host code uses the address that
// hipGetSymbolAddress returns for the device, never the array's name.
constexpr int kNoallocParts = 256;
static __device__ __align__(256) double scratch[kNoallocParts];

constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Resolve the scratch address of `device` (current device at the call).
void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(HFSI_E_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) fail(HFSI_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(p);
}

static double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  double* p = device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
  if (!p) fail(HFSI_E_ORDER, "mass_norm_noalloc: scratch of this device not resolved (hfsi_create)");
  return p;
}

double mass_norm(hfsi_ctx* c, const double* dv) {
  const int nb = 256;
  c->kred.ensure(2 * nb);
  k_massnorm<<<nb, 256, 0, c->stream>>>(c->nb, c->brow.p, c->ncol.p, c->Mval.p, dv, c->kred.p + nb);
  HIP_LAUNCH_CHECK();
  double s2 = device_sum(c, c->kred.p + nb, nb);
  return std::sqrt(s2 > 0 ? s2 : 0.0);
}

}  // namespace hfsi

extern "C" hfsi_status hfsi_assemble_residual_tangent(hfsi_ctx* c, const double* v, double load, double* R,
                                                      hfsi_csr_view* K, hfsi_assembly_info* info) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 3, "assemble_residual_tangent");
  if (!v || !R) fail(HFSI_E_ARG, "assemble: null vector");
  if (info && info->struct_size != sizeof(hfsi_assembly_info)) fail(HFSI_E_ARG, "assemble: struct_size mismatch");
  c->stage = 3;
  hfsi::assemble(c, v, load, R, info);
  c->stage = 4;
  c->H.ready = false;
  hfsi::vanka_invalidate(c);
  if (K) {
    K->n_block_rows = c->n;
    K->n_blocks = c->nb;
    K->block_ptr = c->nptr.p;
    K->block_col = c->ncol.p;
    K->block_val = c->Kval.p;
    K->a_rows = c->A.rows;
    K->a_nnz = (int32_t)c->A.nnz;
    K->a_ptr = c->A.ptr.p;
    K->a_col = c->A.col.p;
    K->a_val = c->A.val.p;
    K->schur_diag = c->schur.p;
  }
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mass_norm(hfsi_ctx* c, const double* dv, double* out) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 1, "mass_norm");
  if (!dv || !out) fail(HFSI_E_ARG, "mass_norm: null pointer");
  *out = hfsi::mass_norm(c, dv);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mass_norm_noalloc(hfsi_ctx* c, const double* dv, double* out) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 1, "mass_norm_noalloc");
  if (!dv || !out) fail(HFSI_E_ARG, "mass_norm_noalloc: null pointer");
  static_assert(kNoallocParts == 256, "k_massnorm_final folds 256 partials with 256 threads");
  double* part = noalloc_scratch(c->device);
  // the grid is the partial count: never more slots than the scratch holds
  k_massnorm<<<kNoallocParts, 256, 0, c->stream>>>(c->nb, c->brow.p, c->ncol.p, c->Mval.p, dv, part);
  HIP_LAUNCH_CHECK();
  k_massnorm_final<<<1, kNoallocParts, 0, c->stream>>>(part, out);
  HIP_LAUNCH_CHECK();
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_export_tangent(hfsi_ctx* c, int32_t* block_ptr, int32_t* block_col, double* block_val,
                                           int32_t* a_ptr, int32_t* a_col, double* a_val, double* schur) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 4, "export_tangent");
  hipStream_t s = c->stream;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  };
  cp(block_ptr, c->nptr.p, sizeof(int) * (c->n + 1));
  cp(block_col, c->ncol.p, sizeof(int) * c->nb);
  cp(block_val, c->Kval.p, sizeof(double) * 16 * (size_t)c->nb);
  cp(a_ptr, c->A.ptr.p, sizeof(int) * (c->A.rows + 1));
  cp(a_col, c->A.col.p, sizeof(int) * c->A.nnz);
  cp(a_val, c->A.val.p, sizeof(double) * c->A.nnz);
  cp(schur, c->schur.p, sizeof(double) * c->n);
  HIP_CHECK(hipStreamSynchronize(s));
  HFSI_ABI_END(c)
}

namespace {

// r_s = c0 d + c1 vel + c2 acc per displacement dof (d from the node-
// interleaved state).
__global__ void k_newmark_history(int n, double c0, double c1, double c2, const double* __restrict__ v,
                                  const double* __restrict__ vel, const double* __restrict__ acc,
                                  double* __restrict__ rs) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3L * n) return;
  const long node = t / 3;
  const int i = (int)(t - 3 * node);
  rs[t] = c0 * v[4 * node + i] + c1 * vel[t] + c2 * acc[t];
}

// a_new = (d_new - d_prev) / (beta dt^2) - vel / (beta dt) - (1-2beta)/(2beta) acc,
// vel += gamma dt a_new + (1-gamma) dt acc, in place.
__global__ void k_newmark_update(int n, double beta, double gamma, double dt, const double* __restrict__ vn,
                                 const double* __restrict__ vp, double* __restrict__ vel, double* __restrict__ acc) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3L * n) return;
  const long node = t / 3;
  const int i = (int)(t - 3 * node);
  const double a0 = acc[t], v0 = vel[t];
  const double a1 = (vn[4 * node + i] - vp[4 * node + i]) / (beta * dt * dt) - v0 / (beta * dt) -
                    (1.0 - 2.0 * beta) / (2.0 * beta) * a0;
  vel[t] = v0 + gamma * dt * a1 + (1.0 - gamma) * dt * a0;
  acc[t] = a1;
}

void require_newmark(hfsi_ctx* c, const char* what) {
  if (!(c->cm > 0.0)) fail(HFSI_E_ORDER, std::string(what) + ": Newmark inertia is off (hfsi_set_newmark)");
}

}  // namespace

extern "C" hfsi_status hfsi_set_newmark(hfsi_ctx* c, double rho, double beta, double gamma, double dt) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 1, "set_newmark");
  if (!(rho >= 0.0) || !std::isfinite(rho)) fail(HFSI_E_ARG, "set_newmark: rho must be finite and >= 0");
  if (rho == 0.0) {
    c->nm_rho = 0.0;
    c->cm = 0.0;
    c->rs.release();
  } else {
    if (!(beta > 0.0 && beta <= 1.0) || !(gamma >= 0.0 && gamma <= 1.0) || !(dt > 0.0) || !std::isfinite(dt))
      fail(HFSI_E_ARG, "set_newmark: need 0 < beta <= 1, 0 <= gamma <= 1, dt > 0");
    const double cm = rho / (beta * dt * dt);
    if (!std::isfinite(cm)) fail(HFSI_E_ARG, "set_newmark: rho / (beta dt^2) overflows");
    c->nm_rho = rho;
    c->nm_beta = beta;
    c->nm_gamma = gamma;
    c->nm_dt = dt;
    c->cm = cm;
    c->rs.zero(3 * (size_t)c->n, c->stream);
  }
  c->keep_valid = false;  // the inertia term changes the tangent
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_newmark_history(hfsi_ctx* c, const double* v_prev, const double* vel,
                                            const double* acc) {
  HFSI_ABI_BEGIN(c)
  require_newmark(c, "newmark_history");
  if (!v_prev || !vel || !acc) fail(HFSI_E_ARG, "newmark_history: null vector");
  const double b = c->nm_beta, dt = c->nm_dt, rho = c->nm_rho;
  k_newmark_history<<<div_up(3L * c->n, 256), 256, 0, c->stream>>>(
      c->n, rho / (b * dt * dt), rho / (b * dt), rho * (1.0 - 2.0 * b) / (2.0 * b), v_prev, vel, acc, c->rs.p);
  HIP_LAUNCH_CHECK();
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_newmark_update(hfsi_ctx* c, const double* v_new, const double* v_prev, double* vel,
                                           double* acc) {
  HFSI_ABI_BEGIN(c)
  require_newmark(c, "newmark_update");
  if (!v_new || !v_prev || !vel || !acc) fail(HFSI_E_ARG, "newmark_update: null vector");
  k_newmark_update<<<div_up(3L * c->n, 256), 256, 0, c->stream>>>(c->n, c->nm_beta, c->nm_gamma, c->nm_dt, v_new,
                                                                  v_prev, vel, acc);
  HIP_LAUNCH_CHECK();
  HFSI_ABI_END(c)
}
