// Learned level-0 interpolation: features, a 64-64-64-27 network in bfloat16
// on MFMA with fp32 accumulation, the masked correction of the classical
// weights, the local ideal-interpolation target and training (fp32
// backward, Adam on fp32 master weights).
//
// Sample: an F point i of level 0 with a non-empty strong C set C_i.
// Features (64): same-component couplings a_ij/a_ii of row i in the 3x3x3
// lattice box of node(i) (slot = (dx+1) + 3(dy+1) + 9(dz+1)), 27 flags for
// j in C_i, log10(kappa)/6 and two material constants, the one-hot
// component, zero padding.  Output slot s corrects w_ij of the C point j that
// sits in slot s.  Target: with F_loc = {i} and the F points of i's component
// among the columns of row i, A[F_loc,F_loc] X = -A[F_loc,C_i], w*_i = row i.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"

using namespace hfsi;

namespace {

constexpr int NIN = 64, NH = 64, NOUTP = 32, NOUT = 27;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NOUTP, NPARAM = OFF_B3 + NOUTP;
constexpr int NWB = NIN * NH + NH * NH + NH * NOUTP;  // bf16 weights (W1|W2|W3)

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int slot_of(const int* lat, int ni, int nj) {
  const int dx = lat[3 * nj] - lat[3 * ni], dy = lat[3 * nj + 1] - lat[3 * ni + 1], dz = lat[3 * nj + 2] - lat[3 * ni + 2];
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return -1;
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

// ------------------------------------------------------------ samples
__global__ void k_sample_flag(int n, const int8_t* __restrict__ state, const int* __restrict__ pptr,
                              int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (state[i] == -1 && pptr[i + 1] > pptr[i]) ? 1 : 0;
}

__global__ void k_sample_rows(int n, const int* __restrict__ flag, const int* __restrict__ sidx, int* __restrict__ rows) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) rows[sidx[i]] = i;
}

__global__ void k_c2f(int n, const int8_t* __restrict__ state, const int* __restrict__ cidx, int* __restrict__ c2f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && state[i] == 1) c2f[cidx[i]] = i;
}

// features, mask, base weights in slot form, and the slot of every P entry:
// the stencil a_ij / a_ii of the same-component neighbours in the 3x3x3
// lattice box, and the P row's entries whose C point lies in the box (the
// mask and base weights; entries outside the box keep their weights)
__global__ void k_features(int ns, const int* __restrict__ rows, const int* __restrict__ ap, const int* __restrict__ ac,
                           const double* __restrict__ av, const int* __restrict__ comp, const int* __restrict__ c2f,
                           const int* __restrict__ pptr, const int* __restrict__ pcol, const double* __restrict__ pval,
                           const int* __restrict__ lat, float mf0, float mf1, float mf2, float* __restrict__ X,
                           float* __restrict__ mask, float* __restrict__ wcl, int* __restrict__ pslot) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ns) return;
  const int i = rows[m], ni = i / 3, c = comp[i];
  // X, mask and wcl arrive zeroed: only the non-zero entries are written
  float* x = X + (size_t)m * NIN;
  float* mk = mask + (size_t)m * NOUTP;
  float* w = wcl + (size_t)m * NOUTP;
  double aii = 0.0;
  for (int e = ap[i]; e < ap[i + 1]; ++e)
    if (ac[e] == i) aii = av[e];
  for (int e = ap[i]; e < ap[i + 1]; ++e) {
    const int j = ac[e];
    if (comp[j] != c) continue;
    const int s = slot_of(lat, ni, j / 3);
    if (s >= 0) x[s] = (float)(av[e] / aii);
  }
  for (int q = pptr[i]; q < pptr[i + 1]; ++q) {
    const int s = slot_of(lat, ni, c2f[pcol[q]] / 3);
    pslot[q] = s;
    if (s >= 0) {
      x[27 + s] = 1.f;
      mk[s] = 1.f;
      w[s] = (float)pval[q];
    }
  }
  x[54] = mf0;
  x[55] = mf1;
  x[56] = mf2;
  x[57 + c] = 1.f;
}

// local ideal interpolation, one wavefront per sample
constexpr int LMAX = 32, CMAX = 27;
__global__ void __launch_bounds__(64)
k_ideal_target(int ns, const int* __restrict__ rows, const int* __restrict__ ap, const int* __restrict__ ac,
               const double* __restrict__ av, const int* __restrict__ comp, const int8_t* __restrict__ state,
               const int* __restrict__ pptr, const int* __restrict__ pcol, const int* __restrict__ c2f,
               const int* __restrict__ lat, const float* __restrict__ wcl, float* __restrict__ wstar,
               int* __restrict__ fail) {
  __shared__ int Fl[LMAX], Cl[CMAX];
  __shared__ double Mx[LMAX][LMAX + CMAX];
  __shared__ int nF, nC, ipos, bad;
  __shared__ double scale;
  const int lane = threadIdx.x;
  for (int m = blockIdx.x; m < ns; m += gridDim.x) {
    const int i = rows[m], ci = comp[i];
    if (lane == 0) {
      int f = 0, cc = 0, ip = -1;
      bad = 0;
      // C points: the columns of the P row
      for (int q = pptr[i]; q < pptr[i + 1]; ++q) {
        if (cc < CMAX) Cl[cc] = c2f[pcol[q]];
        ++cc;
      }
      for (int e = ap[i]; e < ap[i + 1]; ++e) {
        const int j = ac[e];
        if (comp[j] != ci) continue;
        if (j == i || state[j] == -1) {
          if (j == i) ip = f;
          if (f < LMAX) Fl[f] = j;
          ++f;
        }
      }
      if (f > LMAX || cc > CMAX || ip < 0) bad = 1;
      nF = min(f, LMAX);
      nC = min(cc, CMAX);
      ipos = ip;
    }
    __syncthreads();
    const int F = nF, NC = nC, W = LMAX + CMAX;
    for (int t = lane; t < LMAX * W; t += 64) Mx[t / W][t % W] = 0.0;
    __syncthreads();
    // fill the local matrix and the right-hand sides (lanes over entries)
    for (int fi = 0; fi < F; ++fi) {
      const int f = Fl[fi];
      for (int e = ap[f] + lane; e < ap[f + 1]; e += 64) {
        const int g = ac[e];
        for (int t = 0; t < F; ++t)
          if (Fl[t] == g) Mx[fi][t] = av[e];
        for (int t = 0; t < NC; ++t)
          if (Cl[t] == g) Mx[fi][LMAX + t] = -av[e];
      }
    }
    __syncthreads();
    // Gaussian elimination with partial pivoting
    for (int k = 0; k < F && !bad; ++k) {
      if (lane == 0) {
        int p = k;
        double best = fabs(Mx[k][k]);
        for (int r = k + 1; r < F; ++r)
          if (fabs(Mx[r][k]) > best) { best = fabs(Mx[r][k]); p = r; }
        if (best == 0.0) bad = 1;
        if (p != k)
          for (int t = 0; t < W; ++t) {
            const double x = Mx[k][t];
            Mx[k][t] = Mx[p][t];
            Mx[p][t] = x;
          }
      }
      __syncthreads();
      if (bad) break;
      const int r = k + 1 + lane;
      if (r < F) {
        const double fac = Mx[r][k] / Mx[k][k];
        for (int t = k; t < W; ++t) Mx[r][t] -= fac * Mx[k][t];
      }
      __syncthreads();
    }
    // back substitution, one right-hand side per lane
    if (!bad && lane < NC) {
      const int col = LMAX + lane;
      for (int k = F - 1; k >= 0; --k) {
        double s = Mx[k][col];
        for (int t = k + 1; t < F; ++t) s -= Mx[k][t] * Mx[t][col];
        Mx[k][col] = s / Mx[k][k];
      }
    }
    __syncthreads();
    // rescale to the classical row sum (constants are then reproduced as by
    // the classical weights; the local system alone drops outer couplings)
    if (lane == 0 && !bad) {
      double si = 0.0, sc = 0.0;  // over the C points inside the lattice box
      for (int t = 0; t < NC; ++t)
        if (slot_of(lat, i / 3, Cl[t] / 3) >= 0) si += Mx[ipos][LMAX + t];
      for (int t = 0; t < NOUT; ++t) sc += (double)wcl[(size_t)m * NOUTP + t];
      scale = fabs(si) > 1e-12 ? sc / si : 1.0;
    }
    if (lane < NOUTP) wstar[(size_t)m * NOUTP + lane] = 0.f;
    __syncthreads();
    if (bad) {
      if (lane == 0) atomicAdd(fail, 1);
    } else if (lane < NC) {
      const int s = slot_of(lat, i / 3, Cl[lane] / 3);
      if (s >= 0) wstar[(size_t)m * NOUTP + s] = (float)(Mx[ipos][LMAX + lane] * scale);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ network
// 4 wavefronts per block, 16 samples per wavefront, gfx950's
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)+v] and
// B[8(l/16)+v][l%16] (v = 0..7), D[4(l/16)+v][l%16] (v = 0..3).
template <int NJ, bool RELU>
__device__ __forceinline__ void dense_layer(const uint16_t (*in)[NIN + 8], const uint16_t* __restrict__ Wl,
                                            const float* __restrict__ bias, uint16_t (*outb)[NIN + 8],
                                            float* __restrict__ outf, int row0, int M, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int jb = 0; jb < NJ / 16; ++jb) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NIN / 32; ++kb) {
      v8s a, b;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        a[v] = (short)in[lr][32 * kb + 8 * lg + v];
        b[v] = (short)Wl[(32 * kb + 8 * lg + v) * NJ + 16 * jb + lr];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), acc, 0,
                                                     0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * lg + v, col = 16 * jb + lr;
      float y = acc[v] + bias[col];
      if (RELU) {
        y = fmaxf(y, 0.f);
        outb[row][col] = f2bf(y);
      } else if (row0 + row < M) {
        outf[(size_t)(row0 + row) * NOUTP + col] = y;
      }
    }
  }
}

__global__ void __launch_bounds__(256)
k_mlp_fwd(int M, const float* __restrict__ X, const uint16_t* __restrict__ Wb, const float* __restrict__ P,
          float* __restrict__ out, uint16_t* __restrict__ xo, uint16_t* __restrict__ h1o, uint16_t* __restrict__ h2o) {
  __shared__ uint16_t W[NWB];
  __shared__ float bias[NH + NH + NOUTP];
  __shared__ uint16_t act[4][3][16][NIN + 8];
  for (int t = threadIdx.x; t < NWB; t += 256) W[t] = Wb[t];
  for (int t = threadIdx.x; t < NH; t += 256) {
    bias[t] = P[OFF_B1 + t];
    bias[NH + t] = P[OFF_B2 + t];
  }
  for (int t = threadIdx.x; t < NOUTP; t += 256) bias[2 * NH + t] = P[OFF_B3 + t];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + w) * 16;
  for (int t = lane; t < 16 * NIN; t += 64) {
    const int r = t / NIN, k = t % NIN;
    const float v = (row0 + r < M) ? X[(size_t)(row0 + r) * NIN + k] : 0.f;
    act[w][0][r][k] = f2bf(v);
  }
  __syncthreads();
  dense_layer<NH, true>(act[w][0], W, bias, act[w][1], nullptr, row0, M, lane);
  __syncthreads();
  dense_layer<NH, true>(act[w][1], W + NIN * NH, bias + NH, act[w][2], nullptr, row0, M, lane);
  __syncthreads();
  dense_layer<NOUTP, false>(act[w][2], W + NIN * NH + NH * NH, bias + 2 * NH, nullptr, out, row0, M, lane);
  if (xo || h1o || h2o)
    for (int t = lane; t < 16 * NIN; t += 64) {
      const int r = t / NIN, k = t % NIN;
      if (row0 + r >= M) continue;
      const size_t o = (size_t)(row0 + r) * NIN + k;
      if (xo) xo[o] = act[w][0][r][k];
      if (h1o) h1o[o] = act[w][1][r][k];
      if (h2o) h2o[o] = act[w][2][r][k];
    }
}

// P_ij += correction of the slot of j (F rows that are samples)
__global__ void k_apply_correction(int ns, const int* __restrict__ rows, const int* __restrict__ pptr,
                                   const int* __restrict__ pslot, const float* __restrict__ out,
                                   double* __restrict__ pval) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ns) return;
  const int i = rows[m];
  for (int q = pptr[i]; q < pptr[i + 1]; ++q) {
    const int s = pslot[q];
    if (s >= 0) pval[q] += (double)out[(size_t)m * NOUTP + s];
  }
}

__global__ void k_to_bf16(int n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// ------------------------------------------------------------ training
// dout = 2 mask (wcl + out - w*) / count, loss partial sums per block
__global__ void k_loss(int B, const int* __restrict__ idx, const float* __restrict__ out,
                       const float* __restrict__ mask, const float* __restrict__ wcl, const float* __restrict__ wst,
                       float inv_cnt, float* __restrict__ dout, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < B * NOUTP; t += gridDim.x * 256) {
    const int b = t / NOUTP, s = t % NOUTP;
    const size_t g = (size_t)idx[b] * NOUTP + s;
    const float r = (wcl[g] + out[t] - wst[g]) * mask[g];
    dout[t] = 2.f * r * inv_cnt;
    acc += (double)r * r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// number of masked slots of a minibatch (partial sums per block)
__global__ void k_mask_count(int B, const int* __restrict__ idx, const float* __restrict__ mask,
                             double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < B * NOUTP; t += gridDim.x * 256)
    acc += mask[(size_t)idx[t / NOUTP] * NOUTP + t % NOUTP];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Backward products on the fp32 MFMA v_mfma_f32_16x16x4_f32 (the bf16
// activations and weights are exact in fp32, the gradients stay fp32): lane l
// holds A[l%16][l/16] and B[l/16][l%16], D[4(l/16)+v][l%16] (v = 0..3), the
// layout of the bf16 16x16x32 instruction of the forward pass.
//
// dW[k][j] = sum_b act[b][k] d[b][j] (act bf16 with row stride NIN, d with
// row stride J): one wavefront per 16x16 tile of dW and per slice of the
// minibatch; the slices' partial tiles go to part[slice][K*J].
__global__ void __launch_bounds__(64) k_wgrad_mfma(int B, int K, int J, int slices, const uint16_t* __restrict__ act,
                                                   const float* __restrict__ d, float* __restrict__ part) {
  const int tj = J / 16, tiles = (K / 16) * tj;
  const int tile = blockIdx.x % tiles, sl = blockIdx.x / tiles;
  const int kt = tile / tj, jt = tile % tj;
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  const int per = ((B + slices - 1) / slices + 3) / 4 * 4;
  const int b_begin = sl * per, b_end = min(B, b_begin + per);
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int b0 = b_begin; b0 < b_end; b0 += 4) {
    const int b = b0 + lg;
    float a = 0.f, bb = 0.f;
    if (b < b_end) {
      a = bf2f(act[(size_t)b * NIN + 16 * kt + lr]);
      bb = d[(size_t)b * J + 16 * jt + lr];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, acc, 0, 0, 0);
  }
  float* P = part + (size_t)sl * K * J;
#pragma unroll
  for (int v = 0; v < 4; ++v) P[(16 * kt + 4 * lg + v) * J + 16 * jt + lr] = acc[v];
}

// dW[t] = sum over slices of part[slice][t], in slice order
__global__ void k_wgrad_sum(int n, int slices, const float* __restrict__ part, float* __restrict__ dW) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float s = 0.f;
  for (int k = 0; k < slices; ++k) s += part[(size_t)k * n + t];
  dW[t] = s;
}

// db[j] = sum_b d[b][j]: one 256-thread block per j
__global__ void __launch_bounds__(256) k_bgrad(int B, int J, const float* __restrict__ d, float* __restrict__ db) {
  __shared__ float sh[256];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < B; b += 256) s += d[(size_t)b * J + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = sh[0];
}

// dh[b][k] = (sum_j d[b][j] W[k][j]) * (act[b][k] > 0), W bf16 [NH][J]: one
// wavefront per 16 samples x 16 hidden units
__global__ void __launch_bounds__(64) k_hgrad_mfma(int B, int J, const float* __restrict__ d,
                                                   const uint16_t* __restrict__ Wl, const uint16_t* __restrict__ act,
                                                   float* __restrict__ dh) {
  const int kt = blockIdx.x % (NH / 16), bt = blockIdx.x / (NH / 16);
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  const int ba = 16 * bt + lr;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int j0 = 0; j0 < J; j0 += 4) {
    const float a = ba < B ? d[(size_t)ba * J + j0 + lg] : 0.f;
    const float bb = bf2f(Wl[(16 * kt + lr) * J + j0 + lg]);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int b = 16 * bt + 4 * lg + v, k = 16 * kt + lr;
    if (b < B) dh[(size_t)b * NH + k] = bf2f(act[(size_t)b * NIN + k]) > 0.f ? acc[v] : 0.f;
  }
}

__global__ void k_adam(int n, const float* __restrict__ g, float* __restrict__ w, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows(int B, const int* __restrict__ idx, const float* __restrict__ src, int ld,
                              float* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * ld) return;
  const int b = t / ld, k = t % ld;
  dst[t] = src[(size_t)idx[b] * ld + k];
}

}  // namespace

// ================================================================== host side
namespace hfsi {

struct MlpState {
  DevBuf<float> master, m, v, grad;  // fp32 [NPARAM]
  DevBuf<uint16_t> wb;               // bf16 W1|W2|W3
  bool ready = false;
  long step = 0;
  // training set
  long ns = 0, cap = 0;
  DevBuf<float> X, mask, wcl, wst;
};

static MlpState& mlp_state(hfsi_ctx* c) {
  static_assert(sizeof(void*) == 8, "");
  if (!c->mlp_impl) c->mlp_impl = new MlpState();
  return *reinterpret_cast<MlpState*>(c->mlp_impl);
}

void mlp_free(hfsi_ctx* c) {
  delete reinterpret_cast<MlpState*>(c->mlp_impl);
  c->mlp_impl = nullptr;
}

static void refresh_bf16(hfsi_ctx* c, MlpState& S) {
  hipStream_t s = c->stream;
  S.wb.ensure(NWB);
  k_to_bf16<<<div_up(NIN * NH, 256), 256, 0, s>>>(NIN * NH, S.master.p + OFF_W1, S.wb.p);
  k_to_bf16<<<div_up(NH * NH, 256), 256, 0, s>>>(NH * NH, S.master.p + OFF_W2, S.wb.p + NIN * NH);
  k_to_bf16<<<div_up(NH * NOUTP, 256), 256, 0, s>>>(NH * NOUTP, S.master.p + OFF_W3, S.wb.p + NIN * NH + NH * NH);
  HIP_LAUNCH_CHECK();
}

// Samples of level 0 of the current hierarchy: rows, features, mask, classical
// weights and the slot of every P entry.
struct Samples {
  int ns = 0;
  DevBuf<int> rows, pslot, c2f;  // c2f: fine index of every coarse point
  DevBuf<float> X, mask, wcl;
};

static void material_feats(hfsi_ctx* c, float f[3]) {
  const double* m = c->mtab_h.data();
  f[0] = (float)(std::log10(m[3]) / 6.0);
  f[1] = (float)m[1];
  f[2] = (float)(m[0] == 0 ? m[2] : m[4]);
}

static void build_samples(hfsi_ctx* c, Level& L, Samples& S) {
  if (!c->has_lattice) fail(HFSI_E_ARG, "learned interpolation needs lattice coordinates (set_mesh)");
  if (L.n != 3 * c->n) fail(HFSI_E_ORDER, "learned interpolation applies to the assembled A only");
  hipStream_t s = c->stream;
  const int n = L.n;
  DevBuf<int> flag, sidx;
  flag.ensure(n + 1);
  HIP_CHECK(hipMemsetAsync(flag.p + n, 0, sizeof(int), s));
  k_sample_flag<<<div_up(n, 256), 256, 0, s>>>(n, L.state.p, L.P.ptr.p, flag.p);
  HIP_LAUNCH_CHECK();
  sidx.ensure(n + 1);
  S.ns = (int)exclusive_scan(flag.p, sidx.p, n + 1, s);
  S.rows.ensure(std::max(S.ns, 1));
  k_sample_rows<<<div_up(n, 256), 256, 0, s>>>(n, flag.p, sidx.p, S.rows.p);
  HIP_LAUNCH_CHECK();
  S.X.ensure((size_t)std::max(S.ns, 1) * NIN);
  S.mask.ensure((size_t)std::max(S.ns, 1) * NOUTP);
  S.wcl.ensure((size_t)std::max(S.ns, 1) * NOUTP);
  S.pslot.ensure(std::max<int64_t>(L.P.nnz, 1));
  HIP_CHECK(hipMemsetAsync(S.pslot.p, 0xFF, sizeof(int) * std::max<int64_t>(L.P.nnz, 1), s));
  float mf[3];
  material_feats(c, mf);
  S.c2f.ensure(std::max(L.P.cols, 1));
  k_c2f<<<div_up(n, 256), 256, 0, s>>>(n, L.state.p, L.cidx.p, S.c2f.p);
  HIP_LAUNCH_CHECK();
  if (S.ns > 0) {
    HIP_CHECK(hipMemsetAsync(S.X.p, 0, sizeof(float) * (size_t)S.ns * NIN, s));
    HIP_CHECK(hipMemsetAsync(S.mask.p, 0, sizeof(float) * (size_t)S.ns * NOUTP, s));
    HIP_CHECK(hipMemsetAsync(S.wcl.p, 0, sizeof(float) * (size_t)S.ns * NOUTP, s));
    k_features<<<div_up(S.ns, 128), 128, 0, s>>>(S.ns, S.rows.p, L.A.ptr.p, L.A.col.p, L.A.val.p, L.comp.p, S.c2f.p,
                                                 L.P.ptr.p, L.P.col.p, L.P.val.p, c->lattice.p, mf[0], mf[1], mf[2],
                                                 S.X.p, S.mask.p, S.wcl.p, S.pslot.p);
    HIP_LAUNCH_CHECK();
  }
}

static void forward(hfsi_ctx* c, MlpState& W, int M, const float* X, float* out, uint16_t* xo, uint16_t* h1,
                    uint16_t* h2) {
  if (M <= 0) return;
  k_mlp_fwd<<<div_up(M, 64), 256, 0, c->stream>>>(M, X, W.wb.p, W.master.p, out, xo, h1, h2);
  HIP_LAUNCH_CHECK();
}

// Apply the learned correction to level 0's P (called from the AMG set-up).
void learned_correction(hfsi_ctx* c, Level& L) {
  MlpState& W = mlp_state(c);
  if (!W.ready) fail(HFSI_E_ORDER, "learned interpolation requested but no MLP weights are loaded");
  Samples S;
  build_samples(c, L, S);
  if (S.ns == 0) return;
  DevBuf<float> out;
  out.ensure((size_t)S.ns * NOUTP);
  forward(c, W, S.ns, S.X.p, out.p, nullptr, nullptr, nullptr);
  k_apply_correction<<<div_up(S.ns, 256), 256, 0, c->stream>>>(S.ns, S.rows.p, L.P.ptr.p, S.pslot.p, out.p,
                                                                 L.P.val.p);
  HIP_LAUNCH_CHECK();
}

}  // namespace hfsi

// ================================================================== ABI

extern "C" hfsi_status hfsi_mlp_set_weights(hfsi_ctx* c, const float* w) {
  HFSI_ABI_BEGIN(c)
  if (!w) fail(HFSI_E_ARG, "mlp_set_weights: null");
  hfsi::MlpState& S = hfsi::mlp_state(c);
  S.master.upload(w, NPARAM, c->stream);
  S.m.zero(NPARAM, c->stream);
  S.v.zero(NPARAM, c->stream);
  S.step = 0;
  hfsi::refresh_bf16(c, S);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  S.ready = true;
  c->judge.valid = false;
  HFSI_ABI_END(c)
}

namespace {
// 64-bit FNV-1a over a byte string (Fowler, Noll, Vo): offset basis
// 14695981039346656037, prime 1099511628211
uint64_t fnv1a64(const unsigned char* p, size_t n) {
  uint64_t h = 14695981039346656037ull;
  for (size_t k = 0; k < n; ++k) {
    h ^= p[k];
    h *= 1099511628211ull;
  }
  return h;
}
const char kMlpMagic[8] = {'H', 'F', 'S', 'I', 'M', 'L', 'P', '\0'};
}  // namespace

extern "C" hfsi_status hfsi_mlp_load(hfsi_ctx* c, const char* path) {
  HFSI_ABI_BEGIN(c)
  if (!path) fail(HFSI_E_ARG, "mlp_load: null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) fail(HFSI_E_ARG, std::string("mlp_load: cannot open ") + path);
  char magic[8];
  int32_t version = 0, count = 0;
  uint64_t hash = 0;
  std::vector<float> w(NPARAM);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&version, 4, 1, f) == 1 &&
                  std::fread(&count, 4, 1, f) == 1 && count == NPARAM &&
                  std::fread(w.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM && std::fread(&hash, 8, 1, f) == 1;
  const bool trailing = ok && std::fgetc(f) != EOF;
  std::fclose(f);
  if (!ok || std::memcmp(magic, kMlpMagic, 8) != 0)
    fail(HFSI_E_ARG, std::string("mlp_load: ") + path + " is not a weight file of this network");
  if (version != HFSI_MLP_FILE_VERSION) fail(HFSI_E_ARG, "mlp_load: unsupported file version");
  if (trailing) fail(HFSI_E_ARG, "mlp_load: trailing bytes after the hash");
  if (fnv1a64(reinterpret_cast<const unsigned char*>(w.data()), sizeof(float) * NPARAM) != hash)
    fail(HFSI_E_ARG, "mlp_load: parameter hash mismatch (corrupt file)");
  hfsi::MlpState& S = hfsi::mlp_state(c);
  S.master.upload(w.data(), NPARAM, c->stream);
  S.m.zero(NPARAM, c->stream);
  S.v.zero(NPARAM, c->stream);
  S.step = 0;
  hfsi::refresh_bf16(c, S);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  S.ready = true;
  c->judge.valid = false;
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_save(hfsi_ctx* c, const char* path) {
  HFSI_ABI_BEGIN(c)
  if (!path) fail(HFSI_E_ARG, "mlp_save: null path");
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready) fail(HFSI_E_ORDER, "mlp_save: no weights are set");
  std::vector<float> w(NPARAM);
  HIP_CHECK(hipMemcpyAsync(w.data(), S.master.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  const int32_t version = HFSI_MLP_FILE_VERSION, count = NPARAM;
  const uint64_t hash = fnv1a64(reinterpret_cast<const unsigned char*>(w.data()), sizeof(float) * NPARAM);
  FILE* f = std::fopen(path, "wb");
  if (!f) fail(HFSI_E_ARG, std::string("mlp_save: cannot open ") + path);
  bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&version, 4, 1, f) == 1 &&
            std::fwrite(&count, 4, 1, f) == 1 && std::fwrite(w.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM &&
            std::fwrite(&hash, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) fail(HFSI_E_ARG, std::string("mlp_save: cannot write ") + path);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_get_weights(hfsi_ctx* c, float* w) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready || !w) fail(HFSI_E_ORDER, "mlp_get_weights: no weights");
  HIP_CHECK(hipMemcpyAsync(w, S.master.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_forward(hfsi_ctx* c, int32_t m, const float* X, float* out, uint16_t* xo,
                                        uint16_t* h1, uint16_t* h2) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready) fail(HFSI_E_ORDER, "mlp_forward: no weights");
  if (m <= 0 || !X || !out) fail(HFSI_E_ARG, "mlp_forward: bad arguments");
  hipStream_t s = c->stream;
  hfsi::DevBuf<float> dX, dO;
  hfsi::DevBuf<uint16_t> dx, d1, d2;
  dX.upload(X, (size_t)m * NIN, s);
  dO.ensure((size_t)m * NOUTP);
  dx.ensure((size_t)m * NIN);
  d1.ensure((size_t)m * NIN);
  d2.ensure((size_t)m * NIN);
  hfsi::forward(c, S, m, dX.p, dO.p, dx.p, d1.p, d2.p);
  HIP_CHECK(hipMemcpyAsync(out, dO.p, sizeof(float) * m * NOUTP, hipMemcpyDeviceToHost, s));
  if (xo) HIP_CHECK(hipMemcpyAsync(xo, dx.p, sizeof(uint16_t) * m * NIN, hipMemcpyDeviceToHost, s));
  if (h1) HIP_CHECK(hipMemcpyAsync(h1, d1.p, sizeof(uint16_t) * m * NIN, hipMemcpyDeviceToHost, s));
  if (h2) HIP_CHECK(hipMemcpyAsync(h2, d2.p, sizeof(uint16_t) * m * NIN, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  HFSI_ABI_END(c)
}

namespace hfsi {

// loss and gradient of a minibatch idx[0..B) of the training set (device)
static double loss_grad(hfsi_ctx* c, MlpState& S, int B, const int* idx, DevBuf<float>& ws) {
  hipStream_t s = c->stream;
  // workspace: x(f32 gathered), out, dout, dh2, dh1 + bf16 acts
  ws.ensure((size_t)B * (NIN + 3 * NOUTP + 2 * NH) + 1024);
  float* Xb = ws.p;
  float* out = Xb + (size_t)B * NIN;
  float* dout = out + (size_t)B * NOUTP;
  float* dh2 = dout + (size_t)B * NOUTP;
  float* dh1 = dh2 + (size_t)B * NH;
  double* part = reinterpret_cast<double*>(dh1 + (size_t)B * NH + ((size_t)B * NH) % 2);
  DevBuf<uint16_t> acts;
  acts.ensure((size_t)3 * B * NIN);
  uint16_t* xo = acts.p;
  uint16_t* h1 = xo + (size_t)B * NIN;
  uint16_t* h2 = h1 + (size_t)B * NIN;
  k_gather_rows<<<div_up((long)B * NIN, 256), 256, 0, s>>>(B, idx, S.X.p, NIN, Xb);
  HIP_LAUNCH_CHECK();
  forward(c, S, B, Xb, out, xo, h1, h2);
  k_mask_count<<<64, 256, 0, s>>>(B, idx, S.mask.p, part);
  HIP_LAUNCH_CHECK();
  const double inv_cnt = 1.0 / std::max(device_sum(c, part, 64), 1.0);
  k_loss<<<64, 256, 0, s>>>(B, idx, out, S.mask.p, S.wcl.p, S.wst.p, (float)inv_cnt, dout, part);
  HIP_LAUNCH_CHECK();
  S.grad.ensure(NPARAM);
  float* g = S.grad.p;
  const uint16_t* W2 = S.wb.p + NIN * NH;
  const uint16_t* W3 = S.wb.p + NIN * NH + NH * NH;
  // minibatch slices of the weight gradients: about 64 samples each
  const int slices = std::max(1, std::min(32, B / 64));
  DevBuf<float> wpart;
  wpart.ensure((size_t)slices * NH * NH);
  auto wgrad = [&](int K, int J, const uint16_t* act, const float* d, float* dW) {
    k_wgrad_mfma<<<(K / 16) * (J / 16) * slices, 64, 0, s>>>(B, K, J, slices, act, d, wpart.p);
    k_wgrad_sum<<<div_up(K * J, 256), 256, 0, s>>>(K * J, slices, wpart.p, dW);
  };
  const int hblocks = div_up(B, 16) * (NH / 16);
  wgrad(NH, NOUTP, h2, dout, g + OFF_W3);
  k_bgrad<<<NOUTP, 256, 0, s>>>(B, NOUTP, dout, g + OFF_B3);
  k_hgrad_mfma<<<hblocks, 64, 0, s>>>(B, NOUTP, dout, W3, h2, dh2);
  wgrad(NH, NH, h1, dh2, g + OFF_W2);
  k_bgrad<<<NH, 256, 0, s>>>(B, NH, dh2, g + OFF_B2);
  k_hgrad_mfma<<<hblocks, 64, 0, s>>>(B, NH, dh2, W2, h1, dh1);
  wgrad(NIN, NH, xo, dh1, g + OFF_W1);
  k_bgrad<<<NH, 256, 0, s>>>(B, NH, dh1, g + OFF_B1);
  HIP_LAUNCH_CHECK();
  return device_sum(c, part, 64) * inv_cnt;
}

}  // namespace hfsi

extern "C" hfsi_status hfsi_mlp_loss_grad(hfsi_ctx* c, int32_t m, const float* X, const float* mask, const float* wcl,
                                          const float* wstar, float* grad, double* loss) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready) fail(HFSI_E_ORDER, "mlp_loss_grad: no weights");
  if (m <= 0 || !X || !mask || !wcl || !wstar || !grad || !loss) fail(HFSI_E_ARG, "mlp_loss_grad: bad arguments");
  hipStream_t s = c->stream;
  // a temporary training set holding exactly this batch
  hfsi::DevBuf<float> X0, M0, W0, T0;
  std::swap(S.X, X0); std::swap(S.mask, M0); std::swap(S.wcl, W0); std::swap(S.wst, T0);
  S.X.upload(X, (size_t)m * NIN, s);
  S.mask.upload(mask, (size_t)m * NOUTP, s);
  S.wcl.upload(wcl, (size_t)m * NOUTP, s);
  S.wst.upload(wstar, (size_t)m * NOUTP, s);
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  hfsi::DevBuf<int> didx;
  didx.upload(idx.data(), m, s);
  hfsi::DevBuf<float> ws;
  *loss = hfsi::loss_grad(c, S, m, didx.p, ws);
  HIP_CHECK(hipMemcpyAsync(grad, S.grad.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  std::swap(S.X, X0); std::swap(S.mask, M0); std::swap(S.wcl, W0); std::swap(S.wst, T0);
  HFSI_ABI_END(c)
}

// Append the samples of the current (classical) hierarchy to the training set.
namespace hfsi {
namespace {

// keep[t] = 1 when the sample of row rows[t] is drawn: the top 53 bits of
// SplitMix64 output rows[t] of the stream `seed`, as a fraction of 2^53,
// below `fraction`
__global__ void k_sample_keep(int ns, const int* __restrict__ rows, uint64_t seed, double fraction,
                              int* __restrict__ keep) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const double u = (double)(splitmix64(seed, (uint64_t)rows[t]) >> 11) * (1.0 / 9007199254740992.0);
  keep[t] = u < fraction ? 1 : 0;
}

__global__ void k_sample_compact(int ns, const int* __restrict__ keep, const int* __restrict__ kidx,
                                 const int* __restrict__ rows, const float* __restrict__ X,
                                 const float* __restrict__ mask, const float* __restrict__ wcl,
                                 int* __restrict__ rows2, float* __restrict__ X2, float* __restrict__ mask2,
                                 float* __restrict__ wcl2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns || !keep[t]) return;
  const int k = kidx[t];
  rows2[k] = rows[t];
  for (int j = 0; j < NIN; ++j) X2[(size_t)k * NIN + j] = X[(size_t)t * NIN + j];
  for (int j = 0; j < NOUTP; ++j) {
    mask2[(size_t)k * NOUTP + j] = mask[(size_t)t * NOUTP + j];
    wcl2[(size_t)k * NOUTP + j] = wcl[(size_t)t * NOUTP + j];
  }
}

// Append the level-0 samples of the current hierarchy to the training set,
// all of them (fraction >= 1) or those drawn by k_sample_keep.
void collect(hfsi_ctx* c, double fraction, uint64_t seed, int32_t* n_added, int32_t* n_failed) {
  Hierarchy& H = c->H;
  if (!H.ready || H.L.size() < 2) fail(HFSI_E_ORDER, "mlp_collect: needs a hierarchy with at least two levels");
  if (!(fraction > 0.0)) fail(HFSI_E_ARG, "mlp_collect: fraction must be positive");
  MlpState& S = mlp_state(c);
  hipStream_t s = c->stream;
  Level& L = H.L[0];
  Samples smp;
  build_samples(c, L, smp);
  if (fraction < 1.0 && smp.ns > 0) {
    const int n0 = smp.ns;
    DevBuf<int> keep, kidx;
    keep.ensure(n0 + 1);
    kidx.ensure(n0 + 1);
    HIP_CHECK(hipMemsetAsync(keep.p + n0, 0, sizeof(int), s));
    k_sample_keep<<<div_up(n0, 256), 256, 0, s>>>(n0, smp.rows.p, seed, fraction, keep.p);
    HIP_LAUNCH_CHECK();
    const int nk = (int)exclusive_scan(keep.p, kidx.p, n0 + 1, s);
    Samples sub;
    sub.ns = nk;
    sub.rows.ensure(std::max(nk, 1));
    sub.X.ensure((size_t)std::max(nk, 1) * NIN);
    sub.mask.ensure((size_t)std::max(nk, 1) * NOUTP);
    sub.wcl.ensure((size_t)std::max(nk, 1) * NOUTP);
    k_sample_compact<<<div_up(n0, 256), 256, 0, s>>>(n0, keep.p, kidx.p, smp.rows.p, smp.X.p, smp.mask.p, smp.wcl.p,
                                                     sub.rows.p, sub.X.p, sub.mask.p, sub.wcl.p);
    HIP_LAUNCH_CHECK();
    std::swap(smp.rows, sub.rows);
    std::swap(smp.X, sub.X);
    std::swap(smp.mask, sub.mask);
    std::swap(smp.wcl, sub.wcl);
    smp.ns = nk;
    HIP_CHECK(hipStreamSynchronize(s));  // the replaced buffers leave scope
  }
  const long ns = smp.ns;
  if (S.ns + ns > S.cap) {  // grow (keep contents)
    long nc = std::max(2 * S.cap, S.ns + ns + 1024);
    hfsi::DevBuf<float> X, M, Wc, Ws;
    X.ensure(nc * NIN); M.ensure(nc * NOUTP); Wc.ensure(nc * NOUTP); Ws.ensure(nc * NOUTP);
    if (S.ns) {
      HIP_CHECK(hipMemcpyAsync(X.p, S.X.p, sizeof(float) * S.ns * NIN, hipMemcpyDeviceToDevice, s));
      HIP_CHECK(hipMemcpyAsync(M.p, S.mask.p, sizeof(float) * S.ns * NOUTP, hipMemcpyDeviceToDevice, s));
      HIP_CHECK(hipMemcpyAsync(Wc.p, S.wcl.p, sizeof(float) * S.ns * NOUTP, hipMemcpyDeviceToDevice, s));
      HIP_CHECK(hipMemcpyAsync(Ws.p, S.wst.p, sizeof(float) * S.ns * NOUTP, hipMemcpyDeviceToDevice, s));
    }
    std::swap(S.X, X); std::swap(S.mask, M); std::swap(S.wcl, Wc); std::swap(S.wst, Ws);
    S.cap = nc;
  }
  hfsi::DevBuf<int> fl;
  fl.zero(1, s);
  if (ns > 0) {
    HIP_CHECK(hipMemcpyAsync(S.X.p + S.ns * NIN, smp.X.p, sizeof(float) * ns * NIN, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(S.mask.p + S.ns * NOUTP, smp.mask.p, sizeof(float) * ns * NOUTP, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(S.wcl.p + S.ns * NOUTP, smp.wcl.p, sizeof(float) * ns * NOUTP, hipMemcpyDeviceToDevice, s));
    k_ideal_target<<<(int)std::min<long>(ns, 65536), 64, 0, s>>>((int)ns, smp.rows.p, L.A.ptr.p, L.A.col.p, L.A.val.p,
                                                                 L.comp.p, L.state.p, L.P.ptr.p, L.P.col.p,
                                                                 smp.c2f.p, c->lattice.p, smp.wcl.p,
                                                                 S.wst.p + S.ns * NOUTP, fl.p);
    HIP_LAUNCH_CHECK();
  }
  int nf = 0;
  HIP_CHECK(hipMemcpyAsync(&nf, fl.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  S.ns += ns;
  if (n_added) *n_added = (int32_t)ns;
  if (n_failed) *n_failed = nf;
}

}  // namespace
}  // namespace hfsi

extern "C" hfsi_status hfsi_mlp_collect(hfsi_ctx* c, int32_t* n_added, int32_t* n_failed) {
  HFSI_ABI_BEGIN(c)
  hfsi::collect(c, 1.0, 0, n_added, n_failed);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_collect_sampled(hfsi_ctx* c, double fraction, uint64_t seed, int32_t* n_added,
                                                int32_t* n_failed) {
  HFSI_ABI_BEGIN(c)
  if (!(fraction > 0.0 && fraction <= 1.0)) fail(HFSI_E_ARG, "mlp_collect_sampled: fraction in (0, 1]");
  hfsi::collect(c, fraction, seed, n_added, n_failed);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_samples(hfsi_ctx* c, int64_t first, int64_t count, int64_t* total, float* X,
                                        float* mask, float* wcl, float* wstar) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (total) *total = S.ns;
  if (count > 0) {
    if (first < 0 || first + count > S.ns) fail(HFSI_E_ARG, "mlp_samples: range outside the training set");
    hipStream_t s = c->stream;
    auto cp = [&](void* dst, const float* src, int ld) {
      if (dst) HIP_CHECK(hipMemcpyAsync(dst, src + first * ld, sizeof(float) * count * ld, hipMemcpyDeviceToHost, s));
    };
    cp(X, S.X.p, NIN);
    cp(mask, S.mask.p, NOUTP);
    cp(wcl, S.wcl.p, NOUTP);
    cp(wstar, S.wst.p, NOUTP);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_clear(hfsi_ctx* c) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  S.ns = 0;
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_train(hfsi_ctx* c, const hfsi_train_params* prm, const int32_t* order, int64_t n_order,
                                      hfsi_train_info* info) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready) fail(HFSI_E_ORDER, "mlp_train: set initial weights first");
  if (!prm || prm->struct_size != sizeof(hfsi_train_params)) fail(HFSI_E_ARG, "train params: struct_size mismatch");
  if (!order || n_order <= 0 || prm->batch <= 0 || prm->batch > 65536) fail(HFSI_E_ARG, "mlp_train: bad order/batch");
  if (S.ns == 0) fail(HFSI_E_ORDER, "mlp_train: empty training set");
  for (int64_t t = 0; t < n_order; ++t)
    if (order[t] < 0 || order[t] >= S.ns) fail(HFSI_E_ARG, "mlp_train: sample index out of range");
  hipStream_t s = c->stream;
  hfsi::DevBuf<int> dorder;
  dorder.upload(order, n_order, s);
  hfsi::DevBuf<float> ws;
  c->judge.valid = false;
  HIP_CHECK(hipEventRecord(c->ev0, s));
  double first = -1, last = 0;
  int steps = 0;
  const int B = prm->batch;
  for (int64_t t0 = 0; t0 + B <= n_order; t0 += B) {
    const double l = hfsi::loss_grad(c, S, B, dorder.p + t0, ws);
    if (first < 0) first = l;
    last = l;
    ++S.step;
    const float c1 = (float)(1.0 - std::pow(prm->beta1, (double)S.step));
    const float c2 = (float)(1.0 - std::pow(prm->beta2, (double)S.step));
    k_adam<<<div_up(NPARAM, 256), 256, 0, s>>>(NPARAM, S.grad.p, S.master.p, S.m.p, S.v.p, (float)prm->lr,
                                               (float)prm->beta1, (float)prm->beta2, (float)prm->eps, c1, c2);
    HIP_LAUNCH_CHECK();
    hfsi::refresh_bf16(c, S);
    ++steps;
  }
  HIP_CHECK(hipEventRecord(c->ev1, s));
  if (info) {
    info->samples = S.ns;
    info->loss_first = first;
    info->loss_last = last;
    info->steps = steps;
    info->seconds = hfsi::elapsed_ms(c) * 1e-3;
  }
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_mlp_adam_state(hfsi_ctx* c, float* m, float* v, int64_t* step) {
  HFSI_ABI_BEGIN(c)
  hfsi::MlpState& S = hfsi::mlp_state(c);
  if (!S.ready) fail(HFSI_E_ORDER, "mlp_adam_state: no weights");
  if (m) HIP_CHECK(hipMemcpyAsync(m, S.m.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
  if (v) HIP_CHECK(hipMemcpyAsync(v, S.v.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
  if (step) *step = S.step;
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HFSI_ABI_END(c)
}
