// Algebraic multigrid set-up on the displacement block A (the AMG cycles
// that realise Atilde^{-1} in eq. lpre; Galerkin coarse operators as in the
// paper's "AMG methods for the mixed problems").
//
//  * strength, unknown-based: j in S_i iff j != i, comp(j) == comp(i) and
//    -a_ij sgn(a_ii) >= theta m_i, m_i = max_{k != i, same comp} -a_ik sgn(a_ii) > 0
//  * PMIS in synchronous rounds; key_i = (lambda_i << 40) | top 40 bits of
//    SplitMix64(seed, level * 2^40 + i), ties broken by index
//  * modified classical interpolation on same-component strong couplings
//  * R = P^T by counting sort, A_c = R (A P) by a wavefront-per-row hashed
//    sparse product whose accumulation order is fixed (deterministic)
//  * l1-Jacobi diagonal or D^{-1} with a Lanczos estimate for Chebyshev
//  * coarsest level: explicit inverse by Gauss-Jordan with partial pivoting
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "common.hpp"

using namespace hfsi;

namespace {

constexpr int8_t ST_U = 0, ST_C = 1, ST_F = -1;

// ------------------------------------------------------------ strength
// 8 lanes per row; the diagonal (held by one lane) and the row maximum are
// combined exactly, so the flags do not depend on the lane split
__global__ void __launch_bounds__(256)
k_strength(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
           const int* __restrict__ comp, double theta, uint8_t* __restrict__ strong) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (i >= n) return;
  const int lo = ptr[i], hi = ptr[i + 1], ci = comp[i];
  double aii = 0.0;
  for (int e = lo + lane; e < hi; e += 8)
    if (col[e] == i) aii = val[e];
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) aii += __shfl_xor(aii, o, 8);
  const double sg = aii < 0.0 ? -1.0 : 1.0;
  double mi = -INFINITY;
  for (int e = lo + lane; e < hi; e += 8) {
    const int j = col[e];
    if (j != i && comp[j] == ci) mi = fmax(mi, -val[e] * sg);
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) mi = fmax(mi, __shfl_xor(mi, o, 8));
  const double thr = theta * mi;
  for (int e = lo + lane; e < hi; e += 8) {
    const int j = col[e];
    strong[e] = (j != i && comp[j] == ci && mi > 0.0 && -val[e] * sg >= thr) ? 1 : 0;
  }
}

// PMIS kernels: 8 lanes per row
__global__ void __launch_bounds__(256)
k_lambda(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
         int* __restrict__ lam) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (i >= n) return;
  for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 8)
    if (strong[e]) atomicAdd(&lam[col[e]], 1);
}

__global__ void k_pmis_init(int n, const int* __restrict__ lam, uint64_t seed, int level, uint64_t* __restrict__ key,
                            int8_t* __restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64(seed, ((uint64_t)level << 40) | (uint64_t)i) >> 24;
  key[i] = ((uint64_t)lam[i] << 40) | h;
  state[i] = lam[i] == 0 ? ST_F : ST_U;
}

// j beats i when (key_j, j) > (key_i, i)
__global__ void __launch_bounds__(256)
k_pmis_select(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
              const uint64_t* __restrict__ key, const int8_t* __restrict__ state, int* __restrict__ notmax) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (i >= n || state[i] != ST_U) return;
  const uint64_t ki = key[i];
  for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 8) {
    if (!strong[e]) continue;
    const int j = col[e];
    if (state[j] != ST_U) continue;
    const uint64_t kj = key[j];
    if (kj > ki || (kj == ki && j > i)) notmax[i] = 1;
    else notmax[j] = 1;
  }
}

// also clears notmax for the next round
__global__ void k_pmis_mark_c(int n, int* __restrict__ notmax, int8_t* __restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] == ST_U && !notmax[i]) state[i] = ST_C;
  notmax[i] = 0;
}

__global__ void __launch_bounds__(256)
k_pmis_mark_f(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
              int8_t* __restrict__ state, int* __restrict__ remaining) {
  // rows grid-strided; *remaining becomes non-zero if some row stays
  // undecided (one atomic per block: many atomics on one address serialise)
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int lane = threadIdx.x & 7;
  const long groups = ((long)gridDim.x * blockDim.x) >> 3;
  bool left = false;
  for (long i = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 3; i < n; i += groups) {
    if (state[i] != ST_U) continue;  // the 8 lanes of a row move together
    const int hi = ptr[i + 1];
    int found = 0;
    for (int b = ptr[i]; b < hi && !found; b += 8) {
      const int e = b + lane;
      found = e < hi && strong[e] && state[col[e]] == ST_C ? 1 : 0;
#pragma unroll
      for (int o = 4; o > 0; o >>= 1) found |= __shfl_xor(found, o, 8);
    }
    if (lane == 0) {
      if (found) state[i] = ST_F;
      else left = true;
    }
  }
  if (left) any = 1;
  __syncthreads();
  if (threadIdx.x == 0 && any) atomicOr(remaining, 1);
}

__global__ void k_is_c(int n, const int8_t* __restrict__ state, int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = state[i] == ST_C ? 1 : 0;
}

__global__ void k_coarse_comp(int n, const int8_t* __restrict__ state, const int* __restrict__ cidx,
                              const int* __restrict__ comp, int* __restrict__ ccomp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && state[i] == ST_C) ccomp[cidx[i]] = comp[i];
}

// ------------------------------------------------------------ interpolation
__global__ void k_interp_count(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                               const uint8_t* __restrict__ strong, const int8_t* __restrict__ state,
                               int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] == ST_C) { cnt[i] = 1; return; }
  int k = 0;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e)
    if (strong[e] && state[col[e]] == ST_C) ++k;
  cnt[i] = k;
}

__device__ __forceinline__ int find_in(const int* __restrict__ a, int lo, int hi, int key) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Modified classical interpolation of an F row i:
//   w_ij = -(a_ij + sum_{k in F*} a_ik abar_kj / sum_{m in C_i} abar_km)
//          / (a_ii + sum_{weak same comp} a_in + sum_{k in F \ F*} a_ik)
// (C_i the strong C neighbours, F* the strong F neighbours with a non-zero
// denominator, abar_km = a_km where its sign differs from a_kk's, else 0).
// 16 lanes per row: the C_i list and the numerators live in LDS, the rows of
// strong F neighbours are scanned lane-parallel (their sums s are
// tree-reduced; every other sum keeps the row order).
constexpr int CI_MAX = 64;
__global__ void __launch_bounds__(256)
k_interp_fill16(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
                const uint8_t* __restrict__ strong, const int8_t* __restrict__ state, const int* __restrict__ comp,
                const int* __restrict__ cidx, const int* __restrict__ pptr, int* __restrict__ pcol,
                double* __restrict__ pval, int* __restrict__ overflow) {
  __shared__ int s_col[16][CI_MAX];
  __shared__ double s_num[16][CI_MAX];
  const int g = threadIdx.x >> 4, lane = threadIdx.x & 15;
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (i >= n) return;  // whole group
  const int p0 = pptr[i], p1 = pptr[i + 1], nc = p1 - p0;
  if (state[i] == ST_C) {
    if (lane == 0) {
      pcol[p0] = cidx[i];
      pval[p0] = 1.0;
    }
    return;
  }
  if (nc == 0) return;
  if (nc > CI_MAX) {
    if (lane == 0) atomicOr(overflow, 1);
    return;
  }
  int* sc = s_col[g];
  double* sn = s_num[g];
  const int lo = ptr[i], hi = ptr[i + 1], ci = comp[i];
  // strong C neighbours in row order (group prefix over 16-entry chunks)
  double aii = 0.0;
  int q = 0;
  const int gshift = (threadIdx.x & 63) & ~15;
  for (int base = lo; base < hi; base += 16) {
    const int e = base + lane;
    bool isc = false;
    int j = -1;
    if (e < hi) {
      j = col[e];
      if (j == i) aii = val[e];
      isc = strong[e] && state[j] == ST_C;
    }
    const unsigned gm = (unsigned)((__ballot(isc) >> gshift) & 0xFFFFull);
    if (isc) {
      const int at = q + __popc(gm & ((1u << lane) - 1u));
      sc[at] = j;
      sn[at] = 0.0;
    }
    q += __popc(gm);
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) aii += __shfl_xor(aii, o, 16);
  double den = aii;
  for (int e = lo; e < hi; ++e) {
    const int k = col[e];
    if (k == i || comp[k] != ci) continue;
    const double a = val[e];
    if (strong[e] && state[k] == ST_C) {
      if (lane == 0) sn[find_in(sc, 0, nc, k)] += a;
    } else if (strong[e]) {
      const int klo = ptr[k], khi = ptr[k + 1];
      double akk = 0.0, s_neg = 0.0, s_pos = 0.0;
      for (int f = klo + lane; f < khi; f += 16) {
        const int mm = col[f];
        const double v = val[f];
        if (mm == k) akk = v;
        const int pos = find_in(sc, 0, nc, mm);
        if (pos < nc && sc[pos] == mm) {
          if (v < 0.0) s_neg += v;
          else if (v > 0.0) s_pos += v;
        }
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        akk += __shfl_xor(akk, o, 16);
        s_neg += __shfl_xor(s_neg, o, 16);
        s_pos += __shfl_xor(s_pos, o, 16);
      }
      const double sk = akk < 0.0 ? -1.0 : 1.0;
      const double s = sk > 0.0 ? s_neg : s_pos;
      if (s != 0.0) {
        for (int f = klo + lane; f < khi; f += 16) {
          const int mm = col[f];
          const int pos = find_in(sc, 0, nc, mm);
          if (pos < nc && sc[pos] == mm) {
            const double v = val[f];
            if (v * sk < 0.0) sn[pos] += a * v / s;  // distinct columns: one lane per slot
          }
        }
      } else {
        den += a;
      }
    } else {
      den += a;
    }
  }
  for (int t = lane; t < nc; t += 16) {
    pval[p0 + t] = -sn[t] / den;
    pcol[p0 + t] = cidx[sc[t]];
  }
}

// Extended+i interpolation (De Sterck, Falgout, Nolting, Yang 2008) on
// same-component couplings, one wavefront per row.  For an F row i the
// candidate set Chat_i (strong C neighbours of i and of its strong F
// neighbours) is built in an LDS hash table and ranked by column; then
//   w_ij = -(a_ij + sum_{k in F_i} a_ik abar_kj / s_k) / atilde_ii,
//   atilde_ii = a_ii + sum_{weak n not in Chat_i} a_in + sum_k a_ik abar_ki / s_k,
//   s_k = sum_{l in Chat_i + {i}} abar_kl (s_k = 0: a_ik lumped instead).
// The strong F neighbours are taken NG at a time, 64/NG lanes each: within a
// window of 64 entries of row i, neighbour t goes to group t mod NG.  Every
// group keeps its own partial sums, added in group order at the end, so the
// result does not depend on scheduling.  With p_max > 0 a longer row keeps
// its p_max largest |w| (compared in float32: weights equal in exact
// arithmetic stay ties whatever order their fp64 sums ran in; ties to the
// smaller column), rescaled to the full row sum.  FILL = false writes the
// entry count of each row,
// FILL = true the entries (ascending columns).
constexpr int XH = 128;    // hash slots per row
constexpr int XMAX = 96;   // candidates per row
constexpr int XNG = 1;     // strong F neighbours in flight per row (measured fastest of 1/2/4/8)
__device__ __forceinline__ int xh_slot(int key) { return (int)(((unsigned)key * 2654435761u) >> 25); }

// position of the t-th set bit (t < popcount) of a 64-bit mask
__device__ __forceinline__ int nth_set(unsigned long long m, int t) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const int c = __popcll(m & ((1ull << w) - 1ull));
    if (t >= c) {
      t -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// (at most 64 VGPRs, 8 waves per SIMD: a short spill, but more rows in
// flight: the 48^3 set-up 18.0 -> 17.5 ms)
template <bool FILL, int NG>
__global__ void __launch_bounds__(256, 8)
k_extpi(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
        const uint8_t* __restrict__ strong, const int8_t* __restrict__ state, const int* __restrict__ comp,
        const int* __restrict__ cidx, int p_max, int* __restrict__ cnt, const int* __restrict__ pptr,
        int* __restrict__ pcol, double* __restrict__ pval, int* __restrict__ overflow) {
  constexpr int RB = 4;         // rows per block, one wavefront each
  constexpr int SUB = 64 / NG;  // lanes per neighbour
  constexpr int XQ = 256 / SUB; // entries of a neighbour row each lane keeps in registers
  __shared__ int h_key[RB][XH];
  __shared__ int h_rank[RB][XH];
  __shared__ int s_mem[RB][XMAX];   // members in insertion order, then selection ranks
  __shared__ int s_sorted[RB][XMAX];
  __shared__ double s_num[RB][XMAX];
  __shared__ double s_part[RB][NG][XMAX];
  __shared__ int s_cnt[RB];
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane / SUB, sl = lane % SUB;
  const int i = blockIdx.x * RB + g;
  const bool row = i < n && state[i] != ST_C;
  for (int t = lane; t < XH; t += 64) h_key[g][t] = -1;
  if (lane == 0) s_cnt[g] = 0;
  __syncthreads();
  // the strong F neighbours of row i, NG at a time: fn(k, a_ik, row k's
  // first entry, its end) runs on the SUB lanes of one group (called by the
  // whole wavefront)
  auto f_neighbours = [&](auto&& fn) {
    const int lo = ptr[i], hi = ptr[i + 1];
    for (int wb = lo; wb < hi; wb += 64) {
      const int e = wb + lane;
      int kk = 0, kb = 0, ke = 0;
      double aa = 0.0;
      bool isf = false;
      if (e < hi) {
        kk = col[e];
        isf = strong[e] && state[kk] == ST_F;
        aa = val[e];
        if (isf) {
          kb = ptr[kk];
          ke = ptr[kk + 1];
        }
      }
      const unsigned long long fm = __ballot(isf);
      const int nf = __popcll(fm);
      for (int t0 = 0; t0 < nf; t0 += NG) {
        const int t = t0 + grp;
        const int src = t < nf ? nth_set(fm, t) : 0;
        const int k = __shfl(kk, src, 64);
        const double a = __shfl(aa, src, 64);
        const int k0 = __shfl(kb, src, 64), k1 = __shfl(ke, src, 64);
        if (t < nf) fn(k, a, k0, k1);
      }
    }
  };
  // ---- candidates
  if (row) {
    auto insert = [&](int key) {
      int h = xh_slot(key);
      for (int probe = 0; probe < XH; ++probe) {
        const int old = atomicCAS(&h_key[g][h], -1, key);
        if (old == -1) {
          const int at = atomicAdd(&s_cnt[g], 1);
          if (at < XMAX) s_mem[g][at] = key;
          return;
        }
        if (old == key) return;
        h = (h + 1) & (XH - 1);
      }
    };
    const int lo = ptr[i], hi = ptr[i + 1];
    for (int e = lo + lane; e < hi; e += 64) {
      const int j = col[e];
      if (strong[e] && state[j] == ST_C) insert(j);
    }
    f_neighbours([&](int, double, int klo, int khi) {
      for (int f = klo + sl; f < khi; f += SUB) {
        const int mm = col[f];
        if (strong[f] && state[mm] == ST_C) insert(mm);
      }
    });
  }
  __syncthreads();
  const int m = s_cnt[g];
  if (row && m > XMAX && lane == 0) atomicOr(overflow, 1);
  if (!FILL) {
    if (i < n && lane == 0)
      cnt[i] = state[i] == ST_C ? 1 : (m == 0 || m > XMAX ? 0 : (p_max > 0 && m > p_max ? p_max : m));
    return;
  }
  const bool work = row && m > 0 && m <= XMAX;
  // ---- rank by column
  if (work) {
    for (int t = lane; t < m; t += 64) {
      const int key = s_mem[g][t];
      int r = 0;
      for (int u = 0; u < m; ++u) r += s_mem[g][u] < key;
      s_sorted[g][r] = key;
      s_num[g][r] = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) s_part[g][q][r] = 0.0;
      int h = xh_slot(key);
      while (h_key[g][h] != key) h = (h + 1) & (XH - 1);
      h_rank[g][h] = r;
    }
  }
  __syncthreads();
  auto rank_of = [&](int key) -> int {
    int h = xh_slot(key);
    for (int probe = 0; probe < XH; ++probe) {
      const int kk = h_key[g][h];
      if (kk == key) return h_rank[g][h];
      if (kk == -1) return -1;
      h = (h + 1) & (XH - 1);
    }
    return -1;
  };
  double den = 0.0;
  if (work) {
    const int lo = ptr[i], hi = ptr[i + 1], ci = comp[i];
    // row i: direct couplings to Chat_i, weak ones lumped, the diagonal
    double dpart = 0.0;
    for (int e = lo + lane; e < hi; e += 64) {
      const int j = col[e];
      if (comp[j] != ci) continue;
      const double a = val[e];
      if (j == i) {
        dpart += a;
        continue;
      }
      const int r = rank_of(j);
      if (r >= 0) s_num[g][r] += a;
      else if (!(strong[e] && state[j] == ST_F)) dpart += a;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dpart += __shfl_xor(dpart, o, 64);
    den = dpart;
    // strong F neighbours: this group's terms of atilde_ii and of the numerators
    double den_g = 0.0;
    double* part = s_part[g][grp];
    f_neighbours([&](int k, double a_ik, int klo, int khi) {
      double akk = 0.0, s_neg = 0.0, s_pos = 0.0, aki = 0.0;
      bool has_kk = false, has_ki = false;
      int c_r[XQ];  // this lane's entries of row k: rank in Chat_i (or -1) and value
      double c_v[XQ];
#pragma unroll
      for (int q = 0; q < XQ; ++q) {
        c_r[q] = -1;
        c_v[q] = 0.0;
      }
      int q = 0;
      for (int f = klo + sl; f < khi; f += SUB, ++q) {
        const int mm = col[f];
        const double v = val[f];
        if (mm == k) {
          akk = v;
          has_kk = true;
        }
        const int r = mm == i ? -1 : rank_of(mm);
#pragma unroll
        for (int u = 0; u < XQ; ++u)
          if (u == q) {
            c_r[u] = r;
            c_v[u] = v;
          }
        if (mm == i || r >= 0) {
          if (v < 0.0) s_neg += v;
          else if (v > 0.0) s_pos += v;
        }
        if (mm == i) {
          aki = v;
          has_ki = true;
        }
      }
      // a_kk and a_ki sit in one lane each of the group: broadcast them; the
      // two signed sums are reduced
      unsigned long long gmask = ~0ull;
      if constexpr (SUB < 64) gmask = ((1ull << SUB) - 1ull) << (grp * SUB);
      const unsigned long long mkk = __ballot(has_kk) & gmask, mki = __ballot(has_ki) & gmask;
      akk = mkk ? __shfl(akk, __ffsll(mkk) - 1, 64) : 0.0;
      aki = mki ? __shfl(aki, __ffsll(mki) - 1, 64) : 0.0;
#pragma unroll
      for (int o = SUB / 2; o > 0; o >>= 1) {
        s_neg += __shfl_xor(s_neg, o, SUB);
        s_pos += __shfl_xor(s_pos, o, SUB);
      }
      const double sk = akk < 0.0 ? -1.0 : 1.0;
      const double sden = sk > 0.0 ? s_neg : s_pos;
      if (sden == 0.0) {
        den_g += a_ik;
        return;
      }
      q = 0;
      for (int f = klo + sl; f < khi; f += SUB, ++q) {
        int r = -1;
        double v = 0.0;
        if (q < XQ) {
#pragma unroll
          for (int u = 0; u < XQ; ++u)
            if (u == q) {
              r = c_r[u];
              v = c_v[u];
            }
        } else {
          const int mm = col[f];
          r = mm == i ? -1 : rank_of(mm);
          v = val[f];
        }
        if (r < 0) continue;
        if (v * sk < 0.0) part[r] += a_ik * v / sden;  // distinct columns: one lane per slot
      }
      // the coupling back to i counts when its sign is opposite to a_kk's
      const double aki_bar = aki * sk < 0.0 ? aki : 0.0;
      den_g += a_ik * aki_bar / sden;
    });
#pragma unroll
    for (int q = 0; q < NG; ++q) den += __shfl(den_g, q * SUB, 64);
  }
  __syncthreads();
  // ---- weights (in place), selection ranks, output in ascending columns
  if (work)
    for (int t = lane; t < m; t += 64) {
      double v = s_num[g][t];
#pragma unroll
      for (int q = 0; q < NG; ++q) v += s_part[g][q][t];
      s_num[g][t] = -v / den;
    }
  __syncthreads();
  const bool trunc = work && p_max > 0 && m > p_max;
  int* sel = s_mem[g];  // the insertion list is no longer needed
  if (trunc)
    for (int t = lane; t < m; t += 64) {
      const float key = fabsf((float)s_num[g][t]);
      int r = 0;
      for (int u = 0; u < m; ++u) {
        const float ku = fabsf((float)s_num[g][u]);
        r += ku > key || (ku == key && u < t);
      }
      sel[t] = r;
    }
  __syncthreads();
  if (work) {
    double tot = 0.0, kept = 0.0;
    for (int t = lane; t < m; t += 64) {
      tot += s_num[g][t];
      if (trunc && sel[t] < p_max) kept += s_num[g][t];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      tot += __shfl_xor(tot, o, 64);
      kept += __shfl_xor(kept, o, 64);
    }
    const double scale = trunc && kept != 0.0 ? tot / kept : 1.0;
    // pptr == nullptr: rows go to a fixed stride of p_max entries, counts to cnt
    const long p0 = pptr ? (long)pptr[i] : (long)i * p_max;
    if (!pptr && lane == 0) cnt[i] = trunc ? p_max : m;
    for (int t = lane; t < m; t += 64) {
      int pos = t;
      if (trunc) {
        if (sel[t] >= p_max) continue;
        pos = 0;
        for (int u = 0; u < t; ++u) pos += sel[u] < p_max;
      }
      pcol[p0 + pos] = cidx[s_sorted[g][t]];
      pval[p0 + pos] = trunc ? s_num[g][t] * scale : s_num[g][t];
    }
  }
  if (i < n && lane == 0) {
    if (state[i] == ST_C) {
      const long p0 = pptr ? (long)pptr[i] : (long)i * p_max;
      pcol[p0] = cidx[i];
      pval[p0] = 1.0;
      if (!pptr) cnt[i] = 1;
    } else if (!pptr && !work) {
      cnt[i] = 0;
    }
  }
}

// copy rows written at a fixed stride into CSR order
__global__ void k_compact_rows(int n, int stride, const int* __restrict__ ptr, const int* __restrict__ tcol,
                               const double* __restrict__ tval, int* __restrict__ col, double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long src = (long)i * stride;
  for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
    col[q] = tcol[src + q - ptr[i]];
    val[q] = tval[src + q - ptr[i]];
  }
}

// ------------------------------------------------------------ transpose
__global__ void k_count_cols(int n, const int* __restrict__ ptr, const int* __restrict__ col, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) atomicAdd(&cnt[col[e]], 1);
}

__global__ void k_transpose_fill(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                 const double* __restrict__ val, const int* __restrict__ tptr, int* __restrict__ cur,
                                 int* __restrict__ tcol, double* __restrict__ tval) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int J = col[e];
    const int pos = tptr[J] + atomicAdd(&cur[J], 1);
    tcol[pos] = i;
    tval[pos] = val[e];
  }
}

// Rows of a transpose into column order: one wavefront per row; the columns
// of a row are distinct, so each entry's place is the number of smaller
// columns in its row.
__global__ void k_sort_rows(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                            const double* __restrict__ val, int* __restrict__ ocol, double* __restrict__ oval) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int lo = ptr[i], len = ptr[i + 1] - lo;
  for (int p = lane; p < len; p += 64) {
    const int key = col[lo + p];
    int r = 0;
    for (int u = 0; u < len; ++u) r += col[lo + u] < key ? 1 : 0;
    ocol[lo + r] = key;
    oval[lo + r] = val[lo + p];
  }
}

// ------------------------------------------------------------ SpGEMM C = A B
// upper bound of row i of C: sum over k in A_i of nnz(B_k)
// (8 lanes per row)
__global__ void __launch_bounds__(256)
k_spgemm_ub(int n, const int* __restrict__ ap, const int* __restrict__ ac, const int* __restrict__ bp,
            int* __restrict__ ub) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (i >= n) return;
  long s = 0;
  for (int e = ap[i] + lane; e < ap[i + 1]; e += 8) s += bp[ac[e] + 1] - bp[ac[e]];
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 8);
  if (lane == 0) ub[i] = (int)min(s, (long)INT32_MAX);
}

__device__ __forceinline__ unsigned hslot(int key, int mask) { return ((unsigned)key * 2654435761u) & (unsigned)mask; }

// One wavefront per row.  For each k of A_i in ascending order, the lanes
// insert the columns of B_k (distinct within a row of B) into an LDS hash
// table; the value of every C entry is therefore accumulated in ascending k,
// independently of scheduling.  SMALL rows: ub <= TBL*3/4 in the "small"
// pass, the rest in the "large" pass.  NUMERIC = false counts entries.
template <int TBL, bool NUMERIC>
__global__ void __launch_bounds__(64)
k_spgemm(int n, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
         const int* __restrict__ bp, const int* __restrict__ bc, const double* __restrict__ bv,
         const int* __restrict__ sel, int sel_lo, int sel_hi, int* __restrict__ cnt, const int* __restrict__ cp,
         int* __restrict__ cc, double* __restrict__ cv, int* __restrict__ overflow, const int* __restrict__ ubv,
         int ub_min) {
  __shared__ int keys[TBL];
  __shared__ double vals[NUMERIC ? TBL : 1];
  __shared__ int ckeys[NUMERIC ? (TBL * 3) / 4 + 64 : 1];
  __shared__ int ninsert;
  const int lane = threadIdx.x;
  // block b serves rows b, b + G, b + 2G, ... (G = gridDim.x), testing 64 of
  // them at once; `continue` below moves on to the next selected row
  const long G = gridDim.x;
  for (long c0 = 0; blockIdx.x + c0 * G < n; c0 += 64) {
    const long r = blockIdx.x + (c0 + lane) * G;
    unsigned long long pick = __ballot(r < n && sel[r] >= sel_lo && sel[r] <= sel_hi && ubv[r] > ub_min);
    while (pick) {
      const int i = (int)(blockIdx.x + (c0 + __ffsll(pick) - 1) * G);
      pick &= pick - 1;
      const int s = sel[i];
      // table of T = pow2 >= 2 s slots (s = upper bound or exact count of the row)
      int T = 64;
      while (T < 2 * s && T < TBL) T <<= 1;
      const int mask = T - 1;
      for (int t = lane; t < T; t += 64) {
        keys[t] = -1;
        if (NUMERIC) vals[t] = 0.0;
      }
      if (lane == 0) ninsert = 0;
      __syncthreads();
      bool bad = false;
      // the row bounds of B for 64 entries of A_i are fetched at once, then
      // the entries are taken in order
      const int a0 = ap[i], a1 = ap[i + 1];
      for (int base = a0; base < a1; base += 64) {
        int kq0 = 0, kq1 = 0;
        double ka = 0.0;
        if (base + lane < a1) {
          const int kk = ac[base + lane];
          kq0 = bp[kk];
          kq1 = bp[kk + 1];
          if (NUMERIC) ka = av[base + lane];
        }
        const int ne = min(64, a1 - base);
        for (int te = 0; te < ne; ++te) {
          const int q0 = __shfl(kq0, te, 64), q1 = __shfl(kq1, te, 64);
          const double a = NUMERIC ? __shfl(ka, te, 64) : 0.0;
          for (int q = q0 + lane; q < q1; q += 64) {
            const int j = bc[q];
            unsigned h = hslot(j, mask);
            int probes = 0;
            while (true) {
              const int old = atomicCAS(&keys[h], -1, j);
              if (old == -1) {
                if (!NUMERIC) atomicAdd(&ninsert, 1);
                break;
              }
              if (old == j) break;
              h = (h + 1) & mask;
              if (++probes >= T) { bad = true; break; }
            }
            if (NUMERIC && !bad) vals[h] += a * bv[q];
          }
          __syncthreads();
        }
      }
      if (bad) atomicOr(overflow, 1);
      if (!NUMERIC) {
        __syncthreads();
        if (lane == 0) {
          cnt[i] = ninsert;
          if (ninsert > (TBL * 3) / 4) atomicOr(overflow, 4);  // the numeric pass could not hold it
        }
        __syncthreads();
        continue;
      }
      // compact the keys, then place every entry by its rank
      if (lane == 0) ninsert = 0;
      __syncthreads();
      for (int t = lane; t < T; t += 64) {
        const int key = keys[t];
        if (key >= 0) {
          const int pos = atomicAdd(&ninsert, 1);
          if (pos < (TBL * 3) / 4 + 64) ckeys[pos] = key;
        }
      }
      __syncthreads();
      const int nk = ninsert;
      const int base = cp[i];
      if (nk != cp[i + 1] - base || nk > (TBL * 3) / 4 + 64) {
        // a row that cannot be placed gets column 0 / value 0 entries, so
        // that nothing downstream reads an unset column before the flag is
        // checked
        if (lane == 0) atomicOr(overflow, 2);
        for (int t = base + lane; t < cp[i + 1]; t += 64) {
          cc[t] = 0;
          if (cv) cv[t] = 0.0;
        }
        __syncthreads();
        continue;
      }
      for (int t = lane; t < T; t += 64) {
        const int key = keys[t];
        if (key < 0) continue;
        int r = 0;
        for (int u = 0; u < nk; ++u) r += ckeys[u] < key ? 1 : 0;
        cc[base + r] = key;
        cv[base + r] = vals[t];
      }
      __syncthreads();
    }
  }
}

// largest row length of B (wave maximum, one atomic per wavefront)
// (rows grid-strided, one atomic per block)
__global__ void __launch_bounds__(256) k_max_rowlen(int n, const int* __restrict__ ptr, int* __restrict__ out) {
  __shared__ int red[4];
  int len = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    len = max(len, ptr[i + 1] - ptr[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, max(max(red[0], red[1]), max(red[2], red[3])));
}

// Numeric rows of C = A B when no row of B has more than WB entries (B an
// interpolation operator with truncated rows).  One wavefront per row: the
// lanes fetch 64 entries of A_i and their rows of B at once and insert the
// columns into the hash table in parallel, remembering each product's slot;
// the values are then added entry by entry of A_i in ascending order from
// LDS, the order and arithmetic of k_spgemm, without its chain of dependent
// global loads per entry.  Rows whose exact count lies in [sel_lo, sel_hi].
template <int TBL, int WB>
__global__ void __launch_bounds__(64)
k_spgemm_narrow(int n, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
                const int* __restrict__ bp, const int* __restrict__ bc, const double* __restrict__ bv,
                const int* __restrict__ cnt, int sel_lo, int sel_hi, const int* __restrict__ cp,
                int* __restrict__ cc, double* __restrict__ cv, int* __restrict__ overflow) {
  constexpr int CK = (TBL * 3) / 4 + 64;
  __shared__ int keys[TBL];
  __shared__ double vals[TBL];
  __shared__ int f_s[64 * WB];
  __shared__ double f_b[64 * WB];
  __shared__ double f_a[64];
  __shared__ int ckeys[CK];
  __shared__ double cvals[CK];
  __shared__ int ninsert;
  const int lane = threadIdx.x;
  // rows selected 64 at a time as in k_spgemm
  const long G = gridDim.x;
  for (long c0 = 0; blockIdx.x + c0 * G < n; c0 += 64) {
    const long r = blockIdx.x + (c0 + lane) * G;
    unsigned long long pick = __ballot(r < n && cnt[r] >= sel_lo && cnt[r] <= sel_hi);
    while (pick) {
      const int i = (int)(blockIdx.x + (c0 + __ffsll(pick) - 1) * G);
      pick &= pick - 1;
      const int s = cnt[i];
      int T = 64;
      while (T < 2 * s && T < TBL) T <<= 1;
      const int mask = T - 1;
      for (int t = lane; t < T; t += 64) {
        keys[t] = -1;
        vals[t] = 0.0;
      }
      if (lane == 0) ninsert = 0;
      __syncthreads();
      bool bad = false;
      const int a0 = ap[i], a1 = ap[i + 1];
      for (int base = a0; base < a1; base += 64) {
        const int e = base + lane;
        double a = 0.0;
        int qb = 0, ql = 0;
        if (e < a1) {
          const int k = ac[e];
          a = av[e];
          qb = bp[k];
          ql = bp[k + 1] - qb;
        }
        if (ql > WB) {
          bad = true;
          ql = WB;
        }
        int jj[WB];
        double bb[WB];
#pragma unroll
        for (int q = 0; q < WB; ++q)
          if (q < ql) {
            jj[q] = bc[qb + q];
            bb[q] = bv[qb + q];
          }
#pragma unroll
        for (int q = 0; q < WB; ++q) {
          int h = -1;
          if (q < ql) {
            h = (int)hslot(jj[q], mask);
            int probes = 0;
            while (true) {
              const int old = atomicCAS(&keys[h], -1, jj[q]);
              if (old == -1 || old == jj[q]) break;
              h = (h + 1) & mask;
              if (++probes >= T) {
                bad = true;
                h = -1;
                break;
              }
            }
            f_b[lane * WB + q] = bb[q];
          }
          f_s[lane * WB + q] = h;
        }
        f_a[lane] = a;
        __syncthreads();
        const int ne = min(64, a1 - base);
        for (int e2 = 0; e2 < ne; ++e2) {
          if (lane < WB) {
            const int h = f_s[e2 * WB + lane];
            if (h >= 0) vals[h] += f_a[e2] * f_b[e2 * WB + lane];
          }
          __syncthreads();
        }
      }
      if (bad) atomicOr(overflow, 8);
      // compact (key, value) pairs, then place every entry by its rank
      for (int t = lane; t < T; t += 64) {
        const int key = keys[t];
        if (key >= 0) {
          const int pos = atomicAdd(&ninsert, 1);
          if (pos < CK) {
            ckeys[pos] = key;
            cvals[pos] = vals[t];
          }
        }
      }
      __syncthreads();
      const int nk = ninsert;
      const int base = cp[i];
      if (nk != cp[i + 1] - base || nk > CK) {
        // a row that cannot be placed gets column 0 / value 0 entries, so
        // that nothing downstream reads an unset column before the flag is
        // checked
        if (lane == 0) atomicOr(overflow, 2);
        for (int t = base + lane; t < cp[i + 1]; t += 64) {
          cc[t] = 0;
          if (cv) cv[t] = 0.0;
        }
        __syncthreads();
        continue;
      }
      for (int p = lane; p < nk; p += 64) {
        const int key = ckeys[p];
        int r = 0;
        for (int u = 0; u < nk; ++u) r += ckeys[u] < key ? 1 : 0;
        cc[base + r] = key;
        cv[base + r] = cvals[p];
      }
      __syncthreads();
    }
  }
}

// Rows whose product list has ub <= SMAX entries: stage the list in LDS first
// (lanes in parallel: compacted entries of A_i with non-empty B rows, their
// offsets, then every (column, a_ik b_kj) pair), insert the columns into a
// hash table, and accumulate the values entry by entry of A_i in ascending
// order from LDS — the same summation order as the unstaged kernel.
template <int SMAX, bool NUMERIC>
__global__ void __launch_bounds__(64)
k_spgemm_staged(int n, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
                const int* __restrict__ bp, const int* __restrict__ bc, const double* __restrict__ bv,
                const int* __restrict__ ub, int ub_lo, int* __restrict__ cnt, const int* __restrict__ cp,
                int* __restrict__ cc, double* __restrict__ cv, int* __restrict__ overflow) {
  __shared__ int e_k[SMAX], e_off[SMAX + 1];
  __shared__ double e_a[NUMERIC ? SMAX : 1];
  __shared__ int f_j[SMAX];
  __shared__ double f_v[NUMERIC ? SMAX : 1];
  __shared__ int keys[2 * SMAX];
  __shared__ double vals[NUMERIC ? 2 * SMAX : 1];
  __shared__ int ckeys[NUMERIC ? SMAX : 1];
  __shared__ int ne_sh, nk_sh;
  const int lane = threadIdx.x;
  // rows selected 64 at a time as in k_spgemm
  const long G = gridDim.x;
  for (long c0 = 0; blockIdx.x + c0 * G < n; c0 += 64) {
    const long r = blockIdx.x + (c0 + lane) * G;
    unsigned long long pick = __ballot(r < n && ub[r] >= ub_lo && ub[r] <= SMAX);
    while (pick) {
      const int i = (int)(blockIdx.x + (c0 + __ffsll(pick) - 1) * G);
      pick &= pick - 1;
      const int U = ub[i];
      if (U == 0) {
        if (!NUMERIC && lane == 0) cnt[i] = 0;
        continue;
      }
      // 1. compacted entries with their product offsets (wave prefix sums)
      int run_off = 0, run_ne = 0;
      for (int base = ap[i]; base < ap[i + 1]; base += 64) {
        const int e = base + lane;
        int k = 0, len = 0;
        if (e < ap[i + 1]) {
          k = ac[e];
          len = bp[k + 1] - bp[k];
        }
        int inc = len;  // inclusive scan of len over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(inc, o, 64);
          if (lane >= o) inc += y;
        }
        const unsigned long long fm = __ballot(len > 0);
        const int pos = run_ne + __popcll(fm & ((1ull << lane) - 1ull));
        if (len > 0) {
          e_k[pos] = k;
          e_off[pos] = run_off + inc - len;
          if (NUMERIC) e_a[pos] = av[e];
        }
        run_off += __shfl(inc, 63, 64);
        run_ne += __popcll(fm);
      }
      if (lane == 0) {
        e_off[run_ne] = run_off;
        ne_sh = run_ne;
        nk_sh = 0;
      }
      int T = 64;
      while (T < 2 * U) T <<= 1;
      const int mask = T - 1;
      for (int t = lane; t < T; t += 64) {
        keys[t] = -1;
        if (NUMERIC) vals[t] = 0.0;
      }
      __syncthreads();
      const int ne = ne_sh;
      // 2. the (column, value) pairs, lane-parallel over the whole list, four
      //    independent pairs per lane and step so that their loads overlap
      for (int t0 = lane; t0 < U; t0 += 256) {
        int qq[4], ee[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + 64 * u;
          qq[u] = -1;
          if (t < U) {
            int lo = 0, hi = ne - 1;  // last entry with e_off <= t
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (e_off[mid] <= t) lo = mid; else hi = mid - 1;
            }
            ee[u] = lo;
            qq[u] = bp[e_k[lo]] + (t - e_off[lo]);
          }
        }
        int jj[4];
        double vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (qq[u] >= 0) {
            jj[u] = bc[qq[u]];
            if (NUMERIC) vv[u] = bv[qq[u]];
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (qq[u] >= 0) {
            f_j[t0 + 64 * u] = jj[u];
            if (NUMERIC) f_v[t0 + 64 * u] = e_a[ee[u]] * vv[u];
          }
      }
      __syncthreads();
      // 3. hash insertion; f_j[t] becomes the slot of pair t
      bool bad = false;
      for (int t = lane; t < U; t += 64) {
        const int j = f_j[t];
        unsigned h = hslot(j, mask);
        int probes = 0;
        while (true) {
          const int old = atomicCAS(&keys[h], -1, j);
          if (old == -1) {
            if (!NUMERIC) atomicAdd(&nk_sh, 1);
            break;
          }
          if (old == j) break;
          h = (h + 1) & mask;
          if (++probes >= T) { bad = true; break; }
        }
        f_j[t] = (int)h;
      }
      if (bad) atomicOr(overflow, 1);
      __syncthreads();
      if (!NUMERIC) {
        if (lane == 0) cnt[i] = nk_sh;
        __syncthreads();
        continue;
      }
      // 4. accumulate entry by entry (distinct columns within one entry)
      for (int e = 0; e < ne; ++e) {
        for (int t = e_off[e] + lane; t < e_off[e + 1]; t += 64) vals[f_j[t]] += f_v[t];
        __syncthreads();
      }
      // 5. compact the keys and place every entry by its rank
      for (int t = lane; t < T; t += 64) {
        const int key = keys[t];
        if (key >= 0) {
          const int pos = atomicAdd(&nk_sh, 1);
          if (pos < SMAX) ckeys[pos] = key;
        }
      }
      __syncthreads();
      const int nk = nk_sh;
      const int base = cp[i];
      if (nk != cp[i + 1] - base || nk > SMAX) {
        // a row that cannot be placed gets column 0 / value 0 entries, so
        // that nothing downstream reads an unset column before the flag is
        // checked
        if (lane == 0) atomicOr(overflow, 2);
        for (int t = base + lane; t < cp[i + 1]; t += 64) {
          cc[t] = 0;
          if (cv) cv[t] = 0.0;
        }
        __syncthreads();
        continue;
      }
      for (int t = lane; t < T; t += 64) {
        const int key = keys[t];
        if (key < 0) continue;
        int r = 0;
        for (int u = 0; u < nk; ++u) r += ckeys[u] < key ? 1 : 0;
        cc[base + r] = key;
        cv[base + r] = vals[t];
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ smoother data
__global__ void k_l1_diag(int n, const int* __restrict__ ptr, const double* __restrict__ val, double* __restrict__ d,
                          float* __restrict__ d32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) s += fabs(val[e]);
  d[i] = 1.0 / s;
  d32[i] = (float)(1.0 / s);
}

// 1 / a_ii, 8 lanes per row (one lane holds the diagonal; the others add zeros)
__global__ void __launch_bounds__(256)
k_inv_diag(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
           double* __restrict__ d, float* __restrict__ d32) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (i >= n) return;
  double a = 0.0;
  for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 8)
    if (col[e] == i) a = val[e];
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) a += __shfl_xor(a, o, 8);
  if (lane == 0) {
    d[i] = 1.0 / a;
    d32[i] = (float)(1.0 / a);
  }
}

__global__ void k_to_f32(long n, const double* __restrict__ x, float* __restrict__ y) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// ------------------------------------------------------------ coarse inverse
__global__ void k_dense_from_csr(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                 const double* __restrict__ val, double* __restrict__ M) {
  // M is n x 2n: [A | I]
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* row = M + (size_t)i * 2 * n;
  for (int j = 0; j < 2 * n; ++j) row[j] = (j == n + i) ? 1.0 : 0.0;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) row[col[e]] = val[e];
}

// One Gauss-Jordan step on [A | I] (n x 2n, row-major) with partial
// pivoting, from Min into Mout: every block finds the pivot row p of column k
// (largest |value| among rows >= k, ties to the smallest row) in its first
// wavefront, then each thread forms one entry j > k of the step's result:
// row k = Min[p] / Min[p][k]; row r != k = Min[s] - Min[s][k] * row k with
// s = k for r = p (the rows swap), s = r otherwise.  Columns <= k are never
// read again.  Two buffers remove the read-after-write race between the
// pivot row and the rows that use it.
__global__ void __launch_bounds__(256)
k_gj_step(int n, int k, const double* __restrict__ Min, double* __restrict__ Mout, int* __restrict__ singular) {
  __shared__ int s_p;
  __shared__ double s_ip;
  if (*singular) return;
  const size_t w = 2 * (size_t)n;
  if (threadIdx.x < 64) {
    double best = -1.0;
    int bi = k;
    for (int r = k + (int)threadIdx.x; r < n; r += 64) {
      const double a = fabs(Min[(size_t)r * w + k]);
      if (a > best) {
        best = a;
        bi = r;
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
    if (threadIdx.x == 0) {
      s_p = bi;
      s_ip = best > 0.0 ? 1.0 / Min[(size_t)bi * w + k] : 0.0;
      if (!(best > 0.0)) *singular = 1;
    }
  }
  __syncthreads();
  if (s_ip == 0.0) return;
  const int p = s_p;
  const double ip = s_ip;
  const long cols = 2L * n - k - 1;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * cols) return;
  const int r = (int)(t / cols);
  const int j = k + 1 + (int)(t - (long)r * cols);
  const double pk = Min[(size_t)p * w + j] * ip;  // entry j of the normalised pivot row
  if (r == k) {
    Mout[(size_t)k * w + j] = pk;
  } else {
    const int src = r == p ? k : r;
    Mout[(size_t)r * w + j] = Min[(size_t)src * w + j] - Min[(size_t)src * w + k] * pk;
  }
}

__global__ void k_gj_extract(int n, const double* __restrict__ M, double* __restrict__ inv) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  const int r = (int)(t / n), j = (int)(t % n);
  inv[t] = M[(size_t)r * 2 * n + n + j];
}

// ------------------------------------------------------------ Lanczos
__global__ void k_lanczos_init(int n, uint64_t seed, int stream, double* __restrict__ q) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = splitmix64(seed, ((uint64_t)stream << 40) | (uint64_t)i);
  q[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

// w = Dm A (Dm q) - beta q_prev, with Dm = |diag|^{-1/2}
// 16 lanes per row; dm = |diag A|^{-1/2}
__global__ void k_lanczos_apply(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                                const double* __restrict__ val, const double* __restrict__ dm,
                                const double* __restrict__ q, const double* __restrict__ qp,
                                const double* __restrict__ betap, double* __restrict__ w) {
  const double beta = betap ? betap[0] : 0.0;
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int lane = threadIdx.x & 15;
  if (i >= n) return;
  double s = 0.0;
  for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 16) {
    const int j = col[e];
    s += val[e] * (dm[j] * q[j]);
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
  if (lane == 0) w[i] = dm[i] * s - beta * qp[i];
}

// the same step on level 0's 3x3 node blocks (8 lanes per node row, three
// rows each): one column index per nine values instead of one per value
__global__ void k_lanczos_apply_b3(int nn, const int* __restrict__ bptr, const int* __restrict__ bcol,
                                   const double* __restrict__ B, const double* __restrict__ dm,
                                   const double* __restrict__ q, const double* __restrict__ qp,
                                   const double* __restrict__ betap, double* __restrict__ w) {
  const double beta = betap ? betap[0] : 0.0;
  const int node = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (node >= nn) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int e = bptr[node] + lane; e < bptr[node + 1]; e += 8) {
    const int j = 3 * bcol[e];
    const double* v = B + 9 * (size_t)e;
    const double x0 = dm[j] * q[j], x1 = dm[j + 1] * q[j + 1], x2 = dm[j + 2] * q[j + 2];
    s0 += v[0] * x0 + v[1] * x1 + v[2] * x2;
    s1 += v[3] * x0 + v[4] * x1 + v[5] * x2;
    s2 += v[6] * x0 + v[7] * x1 + v[8] * x2;
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 8);
    s1 += __shfl_xor(s1, o, 8);
    s2 += __shfl_xor(s2, o, 8);
  }
  if (lane < 3) {
    const int i = 3 * node + lane;
    const double sv = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
    w[i] = dm[i] * sv - beta * qp[i];
  }
}

__global__ void k_rsqrt_abs(int n, const double* __restrict__ dinv, double* __restrict__ dm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dm[i] = sqrt(fabs(dinv[i]));
}

__global__ void k_dot_partial(int n, const double* __restrict__ x, const double* __restrict__ y,
                              double* __restrict__ part) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) a += x[i] * y[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// y += (-a[0]) x
__global__ void k_axpy_neg_dev(int n, const double* __restrict__ a, const double* __restrict__ x,
                               double* __restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += (-a[0]) * x[i];
}

// y = (1 / d[0]) x
__global__ void k_scale_inv_dev(int n, const double* __restrict__ d, const double* __restrict__ x,
                                double* __restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (1.0 / d[0]) * x[i];
}

// Sum of the 256 block partials of k_dot_partial in one block, in the order
// of the library's two-stage device sum (the same value bit for bit).
// mode 0: out[0] = sum; mode 1: out[0] = sqrt(sum); mode 2 (Lanczos beta of
// step it): b = sqrt(sum), alpha = ab[it]; while not stopped, count the step
// in kst[0] and either stop (b <= 1e-14 |alpha|, kst[1] = 1) or keep
// ab[32 + it] = b.
__global__ void __launch_bounds__(256)
k_dot_finish(const double* __restrict__ part, int mode, double* __restrict__ out, double* __restrict__ ab,
             int* __restrict__ kst, int it) {
  __shared__ double sh[256];
  sh[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    out[0] = sh[0];
  } else if (mode == 1) {
    out[0] = sqrt(sh[0]);
  } else {
    const double b = sqrt(sh[0]);
    if (kst[1]) return;
    kst[0] = it + 1;
    if (b <= 1e-14 * fabs(ab[it])) kst[1] = 1;
    else ab[32 + it] = b;
  }
}

// largest eigenvalue of the symmetric tridiagonal (alpha, beta) by bisection
// on Sturm sequence counts (single thread; k <= 32)
__global__ void k_tridiag_max(const int* __restrict__ kp, const double* __restrict__ alpha,
                              const double* __restrict__ beta, double* __restrict__ out) {
  const int k = kp[0];
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double x = 0.5 * (lo + hi);
    int cnt = 0;  // eigenvalues < x
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
      d = alpha[i] - x - (i > 0 ? b2 / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    if (cnt >= k) hi = x; else lo = x;
    if (hi - lo <= 1e-15 * fmax(fabs(lo), fabs(hi))) break;
  }
  out[0] = 0.5 * (lo + hi);
}


// ----------------------------------------------- padded CSR for the cycle
// per row: number of 4-entry chunks, smallest column, and whether the row
// spans more than 16 bits of columns (1 in wide[r]; its chunks in wc[r])
// (8 lanes per row)
__global__ void __launch_bounds__(256)
k_pack_count(int n, const int* __restrict__ ptr, const int* __restrict__ col, int* __restrict__ chunks,
             int* __restrict__ base, int* __restrict__ wide, int* __restrict__ wc) {
  const int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int lane = threadIdx.x & 7;
  if (r >= n) return;
  const int a = ptr[r], e = ptr[r + 1];
  int mn = INT_MAX, mx = INT_MIN;
  for (int k = a + lane; k < e; k += 8) {
    mn = min(mn, col[k]);
    mx = max(mx, col[k]);
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) {
    mn = min(mn, __shfl_xor(mn, o, 8));
    mx = max(mx, __shfl_xor(mx, o, 8));
  }
  if (lane != 0) return;
  const int nch = (e - a + 3) / 4;
  const bool w = e > a && mx - mn > 65535;
  chunks[r] = nch;
  base[r] = e > a ? mn : 0;
  wide[r] = w ? 1 : 0;
  wc[r] = w ? nch : 0;
}

// wide rows: base = -1 - (index among wide rows), wch = first chunk in c32w
// minus the row's first chunk (widx, wofs: exclusive scans of wide, wc)
__global__ void k_pack_wide(int n, const int* __restrict__ p4, const int* __restrict__ wide,
                            const int* __restrict__ widx, const int* __restrict__ wofs, int* __restrict__ base,
                            int* __restrict__ wch) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || !wide[r]) return;
  base[r] = -1 - widx[r];
  wch[widx[r]] = wofs[r] - p4[r];
}

// one wavefront per row: copy values and columns into the padded layout,
// interleaved for G lanes per row (lanes_for4)
template <class T>
__global__ void k_pack_fill(int n, const int* __restrict__ ptr, const int* __restrict__ col, const T* __restrict__ val,
                            const int* __restrict__ p4, const int* __restrict__ base, const int* __restrict__ wch, int G,
                            uint16_t* __restrict__ c16, int* __restrict__ c32w, T* __restrict__ out) {
  const int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const int a = ptr[r], len = ptr[r + 1] - a;
  const long o = 4L * p4[r];
  const int nch = p4[r + 1] - p4[r];
  const int padded = 4 * nch;
  const int b = base[r];
  const bool wide = b < 0;
  const long ow = wide ? 4L * (p4[r] + wch[-1 - b]) : 0;
  for (int k = lane; k < padded; k += 64) {
    const int ch = k >> 2, t = k & 3;
    const int g0 = ch - ch % G;                // first chunk of the group
    const int q = min(G, nch - g0);            // chunks in the group
    const int src = 4 * g0 + (ch - g0) + q * t;
    const bool real = src < len;
    out[o + k] = real ? val[a + src] : (T)0;
    if (wide) {
      c32w[ow + k] = real ? col[a + src] : col[a];
      c16[o + k] = 0;
    } else {
      const int cc = real ? col[a + src] : b;
      c16[o + k] = (uint16_t)(cc - b);
    }
  }
}
}  // namespace

namespace hfsi {

namespace {

// Largest Ritz value of `steps` Lanczos steps on D^{-1/2} A D^{-1/2}.  The
// recurrence coefficients stay on the device (ab: alpha[32], beta[32], the
// result, the start norm; kst: steps kept, stopped); the host reads only the
// result.
void lanczos_enqueue(hfsi_ctx* c, Level& L, int steps, uint64_t seed, int level, double* out) {
  const int n = L.n;
  // on the aux stream, after the level's operator and diagonal are ready
  hipStream_t s = c->aux;
  HIP_CHECK(hipEventRecord(c->aev[0], c->stream));
  HIP_CHECK(hipStreamWaitEvent(s, c->aev[0], 0));
  StreamTag tag(s);  // the temporaries below stay with the aux stream
  const int nb = 256, g = div_up(n, 256);
  DevBuf<double> q, qp, w, ab, part;
  DevBuf<int> kst;
  q.ensure(n); qp.zero(n, s); w.ensure(n);
  ab.zero(72, s);
  kst.zero(2, s);
  part.ensure(nb);
  k_lanczos_init<<<g, 256, 0, s>>>(n, seed, 1000 + level, q.p);
  HIP_LAUNCH_CHECK();
  k_dot_partial<<<nb, 256, 0, s>>>(n, q.p, q.p, part.p);
  k_dot_finish<<<1, 256, 0, s>>>(part.p, 1, ab.p + 65, ab.p, kst.p, 0);
  k_scale_inv_dev<<<g, 256, 0, s>>>(n, ab.p + 65, q.p, q.p);
  HIP_LAUNCH_CHECK();
  // |diag|^{-1/2} for the scaling, from the smoother's D^{-1} (Chebyshev)
  DevBuf<double> dabs;
  dabs.ensure(n);
  k_rsqrt_abs<<<g, 256, 0, s>>>(n, L.dinv.p, dabs.p);
  HIP_LAUNCH_CHECK();
  const int steps_run = std::min(steps, std::min(n, 32));
  for (int it = 0; it < steps_run; ++it) {
    if (L.bptr)
      k_lanczos_apply_b3<<<div_up((long)L.nbr * 8, 256), 256, 0, s>>>(L.nbr, L.bptr, L.bcol, L.b3d.p, dabs.p, q.p,
                                                                       qp.p, it ? ab.p + 32 + it - 1 : nullptr, w.p);
    else
      k_lanczos_apply<<<div_up((long)n * 16, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, dabs.p, q.p,
                                                                 qp.p, it ? ab.p + 32 + it - 1 : nullptr, w.p);
    k_dot_partial<<<nb, 256, 0, s>>>(n, q.p, w.p, part.p);
    k_dot_finish<<<1, 256, 0, s>>>(part.p, 0, ab.p + it, ab.p, kst.p, it);        // alpha
    k_axpy_neg_dev<<<g, 256, 0, s>>>(n, ab.p + it, q.p, w.p);
    k_dot_partial<<<nb, 256, 0, s>>>(n, w.p, w.p, part.p);
    k_dot_finish<<<1, 256, 0, s>>>(part.p, 2, nullptr, ab.p, kst.p, it);         // beta, stop test
    HIP_LAUNCH_CHECK();
    std::swap(q, qp);  // qp <- q (whole buffers: the blocks may differ in size)
    k_scale_inv_dev<<<g, 256, 0, s>>>(n, ab.p + 32 + it, w.p, q.p);
    HIP_LAUNCH_CHECK();
  }
  k_tridiag_max<<<1, 1, 0, s>>>(kst.p, ab.p, ab.p + 32, out);
  HIP_LAUNCH_CHECK();
}

void transpose(hfsi_ctx* c, const Csr<double>& P, Csr<double>& R) {
  hipStream_t s = c->stream;
  R.rows = P.cols;
  R.cols = P.rows;
  R.nnz = P.nnz;
  DevBuf<int> cnt, cur, tcol;
  DevBuf<double> tval;
  cnt.zero(R.rows + 1, s);
  k_count_cols<<<div_up(P.rows, 256), 256, 0, s>>>(P.rows, P.ptr.p, P.col.p, cnt.p);
  HIP_LAUNCH_CHECK();
  R.ptr.ensure(R.rows + 1);
  exclusive_scan_async(cnt.p, R.ptr.p, R.rows + 1, s);
  cur.zero(R.rows, s);
  tcol.ensure(R.nnz);
  tval.ensure(R.nnz);
  k_transpose_fill<<<div_up(P.rows, 256), 256, 0, s>>>(P.rows, P.ptr.p, P.col.p, P.val.p, R.ptr.p, cur.p, tcol.p,
                                                       tval.p);
  HIP_LAUNCH_CHECK();
  R.col.ensure(R.nnz);
  R.val.ensure(R.nnz);
  k_sort_rows<<<div_up((long)R.rows * 64, 256), 256, 0, s>>>(R.rows, R.ptr.p, tcol.p, tval.p, R.col.p, R.val.p);
  HIP_LAUNCH_CHECK();
}

// C = A B with the structural pattern (no numerical dropping).
// The numeric pass reports overflow into *deferred (checked by the caller
// later: an overflowing row is written with column 0 entries).
// Slot of column j in the sorted window w[0, wl), or -1.
__device__ __forceinline__ int window_slot(const int* w, int wl, int j) {
  int lo = 0, hi = wl - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = w[mid];
    if (v < j) lo = mid + 1;
    else if (v > j) hi = mid - 1;
    else return mid;
  }
  return -1;
}

// Values of C = A B on the pattern of an earlier product of the same two
// patterns (C's row pointer and sorted columns given).  One wavefront per row
// of C; the row's columns are held in LDS windows of W entries (one window
// unless the row is longer).  For every entry a_ik of A_i, in ascending
// order, the products a_ik b_kj are added into the slots of their columns,
// found by binary search: per entry of C the additions are those of the full
// product in the same order and form, so the values are bitwise equal to it.
// NARROW (rows of B with at most WB entries): the lanes take 64 entries of
// A_i and their rows of B at once to find the slots, then add entry by entry
// with WB lanes.  Otherwise the lanes fetch the row bounds of B for 64
// entries of A_i at once and take the entries in order, the lanes over the
// row of B.  A column of B_k inside the window's range but missing from it
// (a pattern that does not belong to these operands) sets bit 16 of *flag.
template <int W, int WB, bool NARROW>
__global__ void __launch_bounds__(64)
k_spgemm_values(int n, const int* __restrict__ ap, const int* __restrict__ ac, const double* __restrict__ av,
                const int* __restrict__ bp, const int* __restrict__ bc, const double* __restrict__ bv,
                const int* __restrict__ cp, const int* __restrict__ cc, double* __restrict__ cv,
                int* __restrict__ flag, int strict) {
  __shared__ int wcol[W];
  __shared__ double wval[W];
  __shared__ int f_s[NARROW ? 64 * WB : 1];
  __shared__ double f_b[NARROW ? 64 * WB : 1];
  __shared__ double f_a[NARROW ? 64 : 1];
  const int lane = threadIdx.x;
  bool bad = false;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int c0 = cp[i], c1 = cp[i + 1];
    const int a0 = ap[i], a1 = ap[i + 1];
    for (int w0 = c0; w0 < c1; w0 += W) {
      const int wl = min(W, c1 - w0);
      for (int t = lane; t < wl; t += 64) {
        wcol[t] = cc[w0 + t];
        wval[t] = 0.0;
      }
      __syncthreads();
      const int jlo = wcol[0], jhi = wcol[wl - 1];
      for (int base = a0; base < a1; base += 64) {
        const int ne = min(64, a1 - base);
        if (NARROW) {
          const int e = base + lane;
          double a = 0.0;
          int qb = 0, ql = 0;
          if (lane < ne) {
            const int k = ac[e];
            a = av[e];
            qb = bp[k];
            ql = bp[k + 1] - qb;
          }
          if (ql > WB) {
            bad = true;
            ql = WB;
          }
#pragma unroll
          for (int q = 0; q < WB; ++q) {
            int h = -1;
            if (q < ql) {
              const int j = bc[qb + q];
              if (j >= jlo && j <= jhi) {
                h = window_slot(wcol, wl, j);
                if (h < 0 && strict) bad = true;
              }
              f_b[lane * WB + q] = bv[qb + q];
            }
            f_s[lane * WB + q] = h;
          }
          f_a[lane] = a;
          __syncthreads();
          for (int e2 = 0; e2 < ne; ++e2) {
            if (lane < WB) {
              const int h = f_s[e2 * WB + lane];
              if (h >= 0) wval[h] += f_a[e2] * f_b[e2 * WB + lane];
            }
            __syncthreads();
          }
        } else {
          int kq0 = 0, kq1 = 0;
          double ka = 0.0;
          if (lane < ne) {
            const int kk = ac[base + lane];
            kq0 = bp[kk];
            kq1 = bp[kk + 1];
            ka = av[base + lane];
          }
          for (int te = 0; te < ne; ++te) {
            const int q0 = __shfl(kq0, te, 64), q1 = __shfl(kq1, te, 64);
            const double a = __shfl(ka, te, 64);
            for (int q = q0 + lane; q < q1; q += 64) {
              const int j = bc[q];
              if (j >= jlo && j <= jhi) {
                const int h = window_slot(wcol, wl, j);
                if (h >= 0) wval[h] += a * bv[q];
                else if (strict) bad = true;
              }
            }
            __syncthreads();
          }
        }
      }
      for (int t = lane; t < wl; t += 64) cv[w0 + t] = wval[t];
      __syncthreads();
    }
  }
  if (__any(bad) && lane == 0) atomicOr(flag, 16);
}

// diagonal entry of every row (0 if the row has none); columns ascending
__global__ void k_diag_of(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                          const double* __restrict__ val, double* __restrict__ dg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = ptr[i], hi = ptr[i + 1] - 1;
  double d = 0.0;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int j = col[mid];
    if (j < i) lo = mid + 1;
    else if (j > i) hi = mid - 1;
    else {
      d = val[mid];
      break;
    }
  }
  dg[i] = d;
}

// Coarse-operator sparsification: an off-diagonal entry is dropped when
// (float)|a_ij| < (float)(eps sqrt(|a_ii| |a_jj|)) (both sides rounded to
// float32 after the fp64 product, square root and scaling, so that entries
// on the threshold in exact arithmetic decide alike whatever the summation
// order of the product); nothing is lumped.  One wavefront per row, 64
// entries per ballot.  FILL = false writes the kept count of row i to cnt[i],
// FILL = true writes the kept entries in order from optr[i].
template <bool FILL>
__global__ void __launch_bounds__(256)
k_drop_small(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
             const double* __restrict__ dg, double eps, int* __restrict__ cnt, const int* __restrict__ optr,
             int* __restrict__ ocol, double* __restrict__ oval) {
  const int i = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;  // uniform per wavefront
  const double di = fabs(dg[i]);
  const int hi = ptr[i + 1];
  int off = FILL ? optr[i] : 0;
  for (int b = ptr[i]; b < hi; b += 64) {
    const int e = b + lane;
    bool keep = false;
    int j = 0;
    double a = 0.0;
    if (e < hi) {
      j = col[e];
      a = val[e];
      keep = j == i || !((float)fabs(a) < (float)(eps * sqrt(di * fabs(dg[j]))));
    }
    const unsigned long long m = __ballot(keep);
    if (FILL && keep) {
      const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
      ocol[pos] = j;
      oval[pos] = a;
    }
    off += __popcll(m);
  }
  if (!FILL && lane == 0) cnt[i] = off;
}

// A <- A without its small off-diagonal entries (k_drop_small), in place of
// the Galerkin product on a coarse level
void drop_small(hfsi_ctx* c, Csr<double>& A, double eps) {
  hipStream_t s = c->stream;
  const int n = A.rows;
  if (n <= 0 || !(eps > 0.0)) return;
  DevBuf<double> dg;
  dg.ensure(n);
  k_diag_of<<<div_up(n, 256), 256, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, dg.p);
  HIP_LAUNCH_CHECK();
  DevBuf<int> cnt;
  cnt.zero(n + 1, s);
  const int grid = div_up((long)n * 64, 256);
  k_drop_small<false><<<grid, 256, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, dg.p, eps, cnt.p, nullptr, nullptr,
                                           nullptr);
  HIP_LAUNCH_CHECK();
  Csr<double> B;
  B.rows = n;
  B.cols = A.cols;
  B.ptr.ensure(n + 1);
  B.nnz = exclusive_scan(cnt.p, B.ptr.p, n + 1, s);
  B.col.ensure(std::max<int64_t>(B.nnz, 1));
  B.val.ensure(std::max<int64_t>(B.nnz, 1));
  k_drop_small<true><<<grid, 256, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, dg.p, eps, nullptr, B.ptr.p, B.col.p,
                                          B.val.p);
  HIP_LAUNCH_CHECK();
  A = std::move(B);
}

// C = A B into the existing pattern of Cm (an earlier product of the same
// patterns, or a sparsified one: strict = false skips the products whose
// column the pattern does not hold); bmax = the longest row of B, as
// returned by spgemm.
void spgemm_values(hfsi_ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& Cm, int bmax,
                   int* deferred, bool strict = true) {
  hipStream_t s = c->stream;
  const int n = A.rows;
  if (Cm.rows != n || Cm.cols != B.cols) fail(HFSI_E_ARG, "sparse product values: pattern of other operands");
  const int grid = std::max(1, std::min(n, 1 << 16));
  if (bmax <= 4)
    k_spgemm_values<512, 4, true><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p,
                                                      Cm.ptr.p, Cm.col.p, Cm.val.p, deferred, strict ? 1 : 0);
  else
    k_spgemm_values<512, 1, false><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p,
                                                       Cm.ptr.p, Cm.col.p, Cm.val.p, deferred, strict ? 1 : 0);
  HIP_LAUNCH_CHECK();
}

int spgemm(hfsi_ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& Cm, int* deferred) {
  hipStream_t s = c->stream;
  const int n = A.rows;
  Cm.rows = n;
  Cm.cols = B.cols;
  DevBuf<int> ub, cnt, flag;
  ub.ensure(n);
  cnt.zero(n + 1, s);
  flag.zero(2, s);  // [0] overflow bits, [1] longest row of B
  k_spgemm_ub<<<div_up((long)n * 8, 256), 256, 0, s>>>(n, A.ptr.p, A.col.p, B.ptr.p, ub.p);
  HIP_LAUNCH_CHECK();
  k_max_rowlen<<<std::min(div_up(B.rows, 256), 1024), 256, 0, s>>>(B.rows, B.ptr.p, flag.p + 1);
  HIP_LAUNCH_CHECK();
  constexpr int TS = 2048, TL = 8192, S1 = 512, S2 = 1024;
  const int grid = std::min(n, 1 << 16);
  // kernels with large LDS tables fit few blocks per CU and serve few rows:
  // fewer blocks, each testing its rows 64 at a time
  const int gridL = std::min(n, 2048);
  // symbolic: staged kernels for product lists up to S2 entries, the
  // unstaged large-table kernel for longer ones
  k_spgemm_staged<S1, false><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, nullptr, B.ptr.p, B.col.p, nullptr, ub.p, 0,
                                                 cnt.p, nullptr, nullptr, nullptr, flag.p);
  k_spgemm_staged<S2, false><<<gridL, 64, 0, s>>>(n, A.ptr.p, A.col.p, nullptr, B.ptr.p, B.col.p, nullptr, ub.p,
                                                 S1 + 1, cnt.p, nullptr, nullptr, nullptr, flag.p);
  k_spgemm<TL, false><<<gridL, 64, 0, s>>>(n, A.ptr.p, A.col.p, nullptr, B.ptr.p, B.col.p, nullptr, ub.p, S2 + 1,
                                          INT32_MAX, cnt.p, nullptr, nullptr, nullptr, flag.p, ub.p, S2);
  HIP_LAUNCH_CHECK();
  Cm.ptr.ensure(n + 1);
  int fl2[2] = {0, 0};  // read in the scan's wait
  int64_t nnz = exclusive_scan(cnt.p, Cm.ptr.p, n + 1, s, flag.p, 2, fl2);
  if (fl2[0]) fail(HFSI_E_CAPACITY, "sparse product: a row exceeds the hash table");
  const int bmax = fl2[1];
  if (nnz > INT32_MAX) fail(HFSI_E_ARG, "sparse product exceeds int32 indexing");
  Cm.nnz = nnz;
  Cm.col.ensure(nnz);
  Cm.val.ensure(nnz);
  // numeric: the unstaged kernels by exact count (measured faster than the
  // staged numeric variant, whose per-row latency chain is no shorter)
  // (a 512-slot table for short rows keeps many more rows in flight per CU)
  if (bmax <= 4) {
    // B with short rows (truncated interpolation): rows up to 384 entries
    k_spgemm_narrow<256, 4><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p, 0,
                                                192, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred);
    k_spgemm_narrow<512, 4><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p, 193,
                                                384, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred);
  } else {
    k_spgemm<256, true><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p, 0,
                                            192, nullptr, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred, ub.p, -1);
    k_spgemm<512, true><<<grid, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p, 193,
                                            384, nullptr, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred, ub.p, -1);
  }
  k_spgemm<TS, true><<<gridL, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p, 385,
                                         TS * 3 / 4, nullptr, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred, ub.p, -1);
  k_spgemm<TL, true><<<gridL, 64, 0, s>>>(n, A.ptr.p, A.col.p, A.val.p, B.ptr.p, B.col.p, B.val.p, cnt.p,
                                         TS * 3 / 4 + 1, TL * 3 / 4, nullptr, Cm.ptr.p, Cm.col.p, Cm.val.p, deferred,
                                         ub.p, -1);
  HIP_LAUNCH_CHECK();
  return bmax;
}

void smoother_data(hfsi_ctx* c, Level& L, const hfsi_amg_params& prm, int level, bool lanczos = true) {
  hipStream_t s = c->stream;
  L.dinv.ensure(L.n);
  L.dinv32.ensure(L.n);
  if (prm.smoother == 0) {
    k_l1_diag<<<div_up(L.n, 256), 256, 0, s>>>(L.n, L.A.ptr.p, L.A.val.p, L.dinv.p, L.dinv32.p);
    HIP_LAUNCH_CHECK();
  } else {
    k_inv_diag<<<div_up((long)L.n * 8, 256), 256, 0, s>>>(L.n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.dinv.p, L.dinv32.p);
    HIP_LAUNCH_CHECK();
    if (lanczos) lanczos_enqueue(c, L, 10, prm.seed, level, c->H.lmax_dev.p + level);  // read when the hierarchy is done
  }
}

void alloc_vectors(Level& L) {
  L.x.ensure(L.n); L.b.ensure(L.n); L.r.ensure(L.n); L.t.ensure(L.n);
  L.xf.ensure(L.n); L.bf.ensure(L.n); L.rf.ensure(L.n); L.tf.ensure(L.n);
}

// padded copy of L.A in the cycle's precision (levels without node blocks);
// same_pattern: L.A has the pattern of the last packing of this level, whose
// chunk layout is kept (values and columns are written again)
void pack_level(hfsi_ctx* c, Level& L, int precision, bool same_pattern = false) {
  hipStream_t s = c->stream;
  Packed4& K = L.pk;
  const int n = L.n;
  if (!same_pattern || K.rows != n) {
    K.rows = n;
    K.p4.ensure(n + 1);
    K.base.ensure(n);
    DevBuf<int> wide, wc, widx;
    wide.ensure(n + 1);
    wc.ensure(n + 1);
    widx.ensure(n + 1);
    k_pack_count<<<div_up((long)n * 8, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, K.p4.p, K.base.p, wide.p, wc.p);
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipMemsetAsync(K.p4.p + n, 0, sizeof(int), s));
    HIP_CHECK(hipMemsetAsync(wide.p + n, 0, sizeof(int), s));
    HIP_CHECK(hipMemsetAsync(wc.p + n, 0, sizeof(int), s));
    K.chunks = exclusive_scan(K.p4.p, K.p4.p, n + 1, s);
    K.nwide = (int)exclusive_scan(wide.p, widx.p, n + 1, s);
    K.wchunks = 0;
    if (K.nwide > 0) {
      K.wchunks = exclusive_scan(wc.p, wc.p, n + 1, s);
      K.wch.ensure(K.nwide);
      k_pack_wide<<<div_up(n, 256), 256, 0, s>>>(n, K.p4.p, wide.p, widx.p, wc.p, K.base.p, K.wch.p);
      HIP_LAUNCH_CHECK();
      K.c32w.ensure(4 * (size_t)K.wchunks);
    } else {
      K.c32w.release();
      K.wch.release();
    }
  }
  const size_t m = 4 * (size_t)K.chunks;
  // keep only the arrays of this precision
  K.c16.ensure(m);
  if (precision == 1) K.v64.release();
  else K.v32.release();
  const int grid = div_up((long)n * 64, 256);
  const int G = lanes_for4(K.chunks, n);
  if (precision == 1) {
    K.v32.ensure(m);
    k_pack_fill<float><<<grid, 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A32.p, K.p4.p, K.base.p, K.wch.p, G, K.c16.p,
                                            K.c32w.p, K.v32.p);
  } else {
    K.v64.ensure(m);
    k_pack_fill<double><<<grid, 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, K.p4.p, K.base.p, K.wch.p, G,
                                             K.c16.p, K.c32w.p, K.v64.p);
  }
  HIP_LAUNCH_CHECK();
  L.packed = true;
}

void copy_csr(hfsi_ctx* c, const Csr<double>& src, Csr<double>& dst) {
  dst.rows = src.rows;
  dst.cols = src.cols;
  dst.nnz = src.nnz;
  dst.ptr.ensure(src.rows + 1);
  dst.col.ensure(src.nnz);
  dst.val.ensure(src.nnz);
  HIP_CHECK(hipMemcpyAsync(dst.ptr.p, src.ptr.p, sizeof(int) * (src.rows + 1), hipMemcpyDeviceToDevice, c->stream));
  HIP_CHECK(hipMemcpyAsync(dst.col.p, src.col.p, sizeof(int) * src.nnz, hipMemcpyDeviceToDevice, c->stream));
  HIP_CHECK(hipMemcpyAsync(dst.val.p, src.val.p, sizeof(double) * src.nnz, hipMemcpyDeviceToDevice, c->stream));
}

__global__ void k_block3(int nb, const double* __restrict__ Kval, double* __restrict__ b3d, float* __restrict__ b3f) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9L * nb) return;
  const long q = t / 9;
  const int rc = (int)(t - 9 * q), r = rc / 3, cc = rc % 3;
  const double v = Kval[16 * q + 4 * r + cc];
  b3d[t] = v;
  b3f[t] = (float)v;
}

__global__ void k_comp_mod3(int n, int* __restrict__ comp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) comp[i] = i % 3;
}

}  // namespace

constexpr int PMIS_BATCH = 3;

namespace {

void set_schedule(Hierarchy& H, const hfsi_amg_params& prm) {
  H.precision = prm.precision;
  H.smoother = prm.smoother;
  H.nu_pre = prm.nu_pre;
  H.nu_post = prm.nu_post;
  H.nu_pre_coarse = prm.nu_pre_coarse;
  H.nu_post_coarse = prm.nu_post_coarse;
  H.cheb_degree = prm.cheb_degree;
  H.cheb_degree_pre = prm.cheb_degree_pre;
  H.cheb_degree_coarse = prm.cheb_degree_coarse;
  H.cheb_ratio = prm.cheb_ratio;
}

// The Lanczos estimates and the coarsest inverse run on the aux stream: a
// set-up joins it before returning, also when it unwinds with an error.
struct AuxJoin {
  hfsi_ctx* c;
  ~AuxJoin() { (void)hipStreamSynchronize(c->aux); }
};

void to_f32_transfer(hfsi_ctx* c, Level& L) {
  hipStream_t s = c->stream;
  L.P32.ensure(L.P.nnz);
  L.R32.ensure(L.R.nnz);
  k_to_f32<<<div_up(L.P.nnz, 256), 256, 0, s>>>(L.P.nnz, L.P.val.p, L.P32.p);
  k_to_f32<<<div_up(L.R.nnz, 256), 256, 0, s>>>(L.R.nnz, L.R.val.p, L.R32.p);
  HIP_LAUNCH_CHECK();
}

// With every level operator final: the coarsest level's explicit inverse (on
// the aux stream while this stream makes the operator copies of the cycle),
// the fp32 and padded copies, then one read of the deferred checks and the
// eigenvalue estimates.  Marks the hierarchy ready.
void finish_hierarchy(hfsi_ctx* c, const hfsi_amg_params& prm, bool same_patterns = false) {
  hipStream_t s = c->stream;
  Hierarchy& H = c->H;
  Level& Lc = H.L.back();
  const int nc = Lc.n;
  H.nc = nc;
  // a coarsest level above the dense limit where the coarsening stalled (no
  // strong couplings, e.g. a mass-dominated operator) is solved by l1-Jacobi
  // sweeps, whose diagonal replaces the (unused) smoother diagonal there;
  // cut by max_levels instead, it is a capacity error
  if (nc > kMaxDenseCoarse && !H.stalled)
    fail(HFSI_E_CAPACITY, "coarsest level larger than 4096 rows (raise max_levels or lower max_coarse)");
  H.coarse_iterative = nc > kMaxDenseCoarse;
  if (H.coarse_iterative) {
    k_l1_diag<<<div_up(nc, 256), 256, 0, s>>>(nc, Lc.A.ptr.p, Lc.A.val.p, Lc.dinv.p, Lc.dinv32.p);
    HIP_LAUNCH_CHECK();
  } else {
    H.coarse_inv.ensure((size_t)nc * nc);
  }
  DevBuf<int> sing;
  sing.zero(1, s);
  HIP_CHECK(hipEventRecord(c->aev[0], s));
  HIP_CHECK(hipStreamWaitEvent(c->aux, c->aev[0], 0));
  if (!H.coarse_iterative) {
    hipStream_t a = c->aux;
    StreamTag tag(a);
    DevBuf<double> M, M2;
    M.ensure(2 * (size_t)nc * nc);
    M2.ensure(2 * (size_t)nc * nc);
    k_dense_from_csr<<<div_up(nc, 256), 256, 0, a>>>(nc, Lc.A.ptr.p, Lc.A.col.p, Lc.A.val.p, M.p);
    HIP_LAUNCH_CHECK();
    // Gauss-Jordan on [A | I]: one launch per pivot, alternating buffers
    double* gin = M.p;
    double* gout = M2.p;
    for (int k = 0; k < nc; ++k) {
      const long work = (long)nc * (2L * nc - k - 1);
      k_gj_step<<<div_up(work, 256), 256, 0, a>>>(nc, k, gin, gout, sing.p);
      std::swap(gin, gout);
    }
    k_gj_extract<<<div_up((long)nc * nc, 256), 256, 0, a>>>(nc, gin, H.coarse_inv.p);
    HIP_LAUNCH_CHECK();
  }
  // fp32 operator copies
  if (prm.precision == 1)
    for (auto& L : H.L) {
      L.A32.ensure(L.A.nnz);
      k_to_f32<<<div_up(L.A.nnz, 256), 256, 0, s>>>(L.A.nnz, L.A.val.p, L.A32.p);
      HIP_LAUNCH_CHECK();
    }
  // padded operator copies for the smoother and residual
  for (auto& L : H.L) {
    L.packed = false;
    if (!L.bptr) pack_level(c, L, prm.precision, same_patterns);
  }
  // join the aux stream, then read the singularity flag and the estimates
  HIP_CHECK(hipEventRecord(c->aev[1], c->aux));
  HIP_CHECK(hipStreamWaitEvent(s, c->aev[1], 0));
  const int nl = (int)H.L.size();
  double lm[32] = {0};
  int sg = 0, sf = 0;
  HIP_CHECK(hipMemcpyAsync(&sg, sing.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&sf, H.setup_flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
  if (prm.smoother == 1) HIP_CHECK(hipMemcpyAsync(lm, H.lmax_dev.p, sizeof(double) * nl, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (sf & 16) fail(HFSI_E_HIP, "sparse product values: a product column is missing from the kept pattern");
  if (sf) fail(HFSI_E_CAPACITY, "sparse product: a row has more than 6144 entries or overflowed its table");
  if (sg) fail(HFSI_E_BREAKDOWN, "coarsest AMG operator is singular");
  for (int l = 0; l < nl; ++l) H.L[l].lmax = prm.smoother == 1 ? lm[l] : 0.0;
  H.ready = true;
}

void fill_info(const Hierarchy& H, hfsi_amg_info* info, int rounds, double rho) {
  if (!info) return;
  info->levels = (int)H.L.size();
  double nnz0 = (double)H.L[0].A.nnz, rows0 = (double)H.L[0].n, sn = 0, sr = 0;
  for (size_t l = 0; l < H.L.size() && l < 32; ++l) {
    info->rows[l] = H.L[l].n;
    info->nnz[l] = H.L[l].A.nnz;
    sn += (double)H.L[l].A.nnz;
    sr += H.L[l].n;
  }
  info->op_complexity = sn / nnz0;
  info->grid_complexity = sr / rows0;
  info->pmis_rounds = rounds;
  info->rho = rho;
  info->rho_classical = -1.0;
  info->krylov_rho = -1.0;
  info->krylov_rho_classical = -1.0;
  info->learned_used = H.learned;
}

}  // namespace

// C = A B on the structural product pattern (overflow bits into *deferred)
int sparse_product(hfsi_ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& Cm, int* deferred) {
  return spgemm(c, A, B, Cm, deferred);
}

// Build levels 1.. from level 0 (whose A and comp are already set), with no
// judge: the learned level-0 correction is applied when prm.interp == 1.
void build_levels(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info) {
  hipStream_t s = c->stream;
  Hierarchy& H = c->H;
  H.ready = false;
  H.reusable = false;
  H.stalled = false;
  set_schedule(H, prm);
  AuxJoin aux_join{c};
  H.lmax_dev.ensure(32);
  H.setup_flags.zero(1, s);
  int rounds_total = 0;
  DevBuf<int> lam, notmax, flag, rem;
  DevBuf<uint64_t> key;
  rem.ensure(PMIS_BATCH);
  for (int l = 0;; ++l) {
    Level& L = H.L[l];
    const int n = L.n;
    alloc_vectors(L);
    // the level's Lanczos estimate goes to the aux stream once this stream
    // has the level's first set-up kernels (their run covers the host's
    // enqueueing of the estimate's launches)
    smoother_data(c, L, prm, l, false);
    const bool cheb = prm.smoother == 1;
    if (n <= prm.max_coarse || l + 1 >= prm.max_levels || l + 1 >= 32) {
      if (cheb) lanczos_enqueue(c, L, 10, prm.seed, l, H.lmax_dev.p + l);
      break;
    }
    // strength and PMIS
    L.strong.ensure(L.A.nnz);
    k_strength<<<div_up((long)n * 8, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.comp.p, prm.strength_theta,
                                              L.strong.p);
    HIP_LAUNCH_CHECK();
    lam.zero(n, s);
    k_lambda<<<div_up((long)n * 8, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.strong.p, lam.p);
    HIP_LAUNCH_CHECK();
    key.ensure(n);
    L.state.ensure(n);
    k_pmis_init<<<div_up(n, 256), 256, 0, s>>>(n, lam.p, prm.seed, l, key.p, L.state.p);
    HIP_LAUNCH_CHECK();
    if (cheb) lanczos_enqueue(c, L, 10, prm.seed, l, H.lmax_dev.p + l);
    // PMIS rounds, PMIS_BATCH per host read of the undecided flags; rounds
    // after the last undecided point is gone change nothing
    notmax.zero(n, s);
    for (int round = 0;; round += PMIS_BATCH) {
      if (round > n + 1) fail(HFSI_E_HIP, "PMIS did not terminate");
      HIP_CHECK(hipMemsetAsync(rem.p, 0, sizeof(int) * PMIS_BATCH, s));
      for (int k = 0; k < PMIS_BATCH; ++k) {
        k_pmis_select<<<div_up((long)n * 8, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.strong.p, key.p, L.state.p, notmax.p);
        HIP_LAUNCH_CHECK();
        k_pmis_mark_c<<<div_up(n, 256), 256, 0, s>>>(n, notmax.p, L.state.p);
        HIP_LAUNCH_CHECK();
        k_pmis_mark_f<<<std::min(div_up((long)n * 8, 256), 2048), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.strong.p,
                                                                               L.state.p, rem.p + k);
        HIP_LAUNCH_CHECK();
      }
      int left[PMIS_BATCH];
      HIP_CHECK(hipMemcpyAsync(left, rem.p, sizeof(left), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      int k = 0;
      while (k < PMIS_BATCH && left[k] != 0) ++k;
      if (k < PMIS_BATCH) {
        rounds_total += k + 1;
        break;
      }
      rounds_total += PMIS_BATCH;
    }
    // coarse numbering
    flag.ensure(n + 1);
    HIP_CHECK(hipMemsetAsync(flag.p + n, 0, sizeof(int), s));
    k_is_c<<<div_up(n, 256), 256, 0, s>>>(n, L.state.p, flag.p);
    HIP_LAUNCH_CHECK();
    L.cidx.ensure(n + 1);
    const int nc = (int)exclusive_scan(flag.p, L.cidx.p, n + 1, s);
    if (nc == 0 || nc > 0.9 * n) {
      H.stalled = true;
      break;
    }
    // interpolation
    DevBuf<int> cnt;
    cnt.ensure(n + 1);
    HIP_CHECK(hipMemsetAsync(cnt.p + n, 0, sizeof(int), s));
    const bool extpi = prm.interp_kind == 1;
    DevBuf<int> ovf;
    ovf.zero(1, s);
    // with truncation the rows have at most p_max entries: one pass writes
    // counts and entries at a fixed stride, compacted after the scan
    const bool strided = extpi && prm.p_max > 0;
    DevBuf<int> tcol;
    DevBuf<double> tval;
    if (strided) {
      tcol.ensure((size_t)n * prm.p_max);
      tval.ensure((size_t)n * prm.p_max);
      k_extpi<true, XNG><<<div_up(n, 4), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.strong.p,
                                                               L.state.p, L.comp.p, L.cidx.p, prm.p_max, cnt.p,
                                                               nullptr, tcol.p, tval.p, ovf.p);
    } else if (extpi) {
      k_extpi<false, XNG><<<div_up(n, 4), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.strong.p,
                                                                L.state.p, L.comp.p, L.cidx.p, prm.p_max, cnt.p,
                                                                nullptr, nullptr, nullptr, ovf.p);
    } else {
      k_interp_count<<<div_up(n, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.strong.p, L.state.p, cnt.p);
    }
    HIP_LAUNCH_CHECK();
    L.P.rows = n;
    L.P.cols = nc;
    L.P.ptr.ensure(n + 1);
    int o = 0;  // overflow of the single strided pass, read in the scan's wait
    L.P.nnz = strided ? exclusive_scan(cnt.p, L.P.ptr.p, n + 1, s, ovf.p, 1, &o)
                      : exclusive_scan(cnt.p, L.P.ptr.p, n + 1, s);
    if (o) fail(HFSI_E_CAPACITY, "extended interpolation: a row has more than 96 candidate C points");
    L.P.col.ensure(L.P.nnz);
    L.P.val.ensure(L.P.nnz);
    if (strided) {
      k_compact_rows<<<div_up(n, 256), 256, 0, s>>>(n, prm.p_max, L.P.ptr.p, tcol.p, tval.p, L.P.col.p, L.P.val.p);
      HIP_LAUNCH_CHECK();
    } else {
      if (extpi)
        k_extpi<true, XNG><<<div_up(n, 4), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.strong.p,
                                                                 L.state.p, L.comp.p, L.cidx.p, prm.p_max, nullptr,
                                                                 L.P.ptr.p, L.P.col.p, L.P.val.p, ovf.p);
      else
        k_interp_fill16<<<div_up((long)n * 16, 256), 256, 0, s>>>(n, L.A.ptr.p, L.A.col.p, L.A.val.p, L.strong.p,
                                                                   L.state.p, L.comp.p, L.cidx.p, L.P.ptr.p,
                                                                   L.P.col.p, L.P.val.p, ovf.p);
      HIP_LAUNCH_CHECK();
      HIP_CHECK(hipMemcpyAsync(&o, ovf.p, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      if (o)
        fail(HFSI_E_CAPACITY, extpi ? "extended interpolation: a row has more than 96 candidate C points"
                                    : "interpolation: a row has more than 64 strong C neighbours");
    }
    if (l == 0 && prm.interp == 1) learned_correction(c, L);
    transpose(c, L.P, L.R);
    // Galerkin product
    L.p_rowmax = spgemm(c, L.A, L.P, L.AP, H.setup_flags.p);
    H.L.emplace_back();
    Level& Lc = H.L.back();
    Level& Lf = H.L[l];  // reference may move with emplace_back
    Lf.ap_rowmax = spgemm(c, Lf.R, Lf.AP, Lc.A, H.setup_flags.p);
    drop_small(c, Lc.A, prm.drop_tol);
    Lc.n = nc;
    Lc.comp.ensure(nc);
    k_coarse_comp<<<div_up(n, 256), 256, 0, s>>>(n, Lf.state.p, Lf.cidx.p, Lf.comp.p, Lc.comp.p);
    HIP_LAUNCH_CHECK();
    if (prm.precision == 1) to_f32_transfer(c, Lf);
  }
  H.learned = prm.interp == 1 ? 1 : 0;
  H.drop_tol = prm.drop_tol;
  finish_hierarchy(c, prm);
  fill_info(H, info, rounds_total, -1.0);
}

// The hierarchy with the judge of the learned interpolation: the learned
// level-0 rows are kept only if the convergence factor rho of the V-cycle
// (10 stationary cycles from the SplitMix64 vector of seed 777) is at most
// fallback_rho and, with judge_classical > 0, the learned hierarchy solves
// at least as fast as the classical one: on a hierarchy of the assembled
// tangent the rate (||r_k|| / ||r_0||)^(1/k) of kJudgeSteps FGMRES steps on
// K x = b with P_L (b the SplitMix64 vector of seed 777, fixed dofs zeroed)
// is compared, on one of a caller matrix the V-cycle factors; otherwise the
// classical hierarchy is built.  judge_classical = 2 compares on the first
// set-up of a mesh, boundary set, material table, weight set and parameter
// set and keeps the verdict for the later set-ups (the learned rows follow
// the local stencils, which the tangents of one problem share); 1 compares
// on every set-up.
constexpr int kJudgeSteps = 20;

void build_hierarchy(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info) {
  Hierarchy& H = c->H;
  if (prm.interp != 1) {
    build_levels(c, prm, info);
    return;
  }
  hfsi_amg_params cl = prm;
  cl.interp = 0;
  auto& J = c->judge;
  const bool tangent = H.L[0].bptr != nullptr && c->stage >= 4;
  const bool cached = prm.judge_classical == 2 && J.valid && std::memcmp(&J.prm, &prm, sizeof(prm)) == 0;
  auto report = [&](double rho, double rho_c, double kl, double kc, bool keep) {
    if (!info) return;
    info->rho = rho;
    info->rho_classical = rho_c;
    info->krylov_rho = kl;
    info->krylov_rho_classical = kc;
    info->learned_used = keep ? 1 : 0;
  };
  if (cached && !J.learned_wins) {
    H.L.resize(1);
    build_levels(c, cl, info);
    report(J.rho_learned, J.rho_classical, J.krylov_learned, J.krylov_classical, false);
    return;
  }
  build_levels(c, prm, info);
  const double rho = convergence_factor(c, 10, 777);
  double rho_c = cached ? J.rho_classical : -1.0;
  double kl = cached ? J.krylov_learned : -1.0, kc = cached ? J.krylov_classical : -1.0;
  bool keep = rho <= prm.fallback_rho;  // false for NaN
  if (keep && prm.judge_classical > 0 && !cached) {
    if (tangent) kl = krylov_factor(c, kJudgeSteps, 777);
    H.L.resize(1);
    build_levels(c, cl, info);
    rho_c = convergence_factor(c, 10, 777);
    if (tangent) {
      kc = krylov_factor(c, kJudgeSteps, 777);
      keep = kl <= kc;
    } else {
      keep = rho <= rho_c;
    }
    if (keep) {
      H.L.resize(1);
      build_levels(c, prm, info);
    }
    if (prm.judge_classical == 2) {
      J.valid = true;
      J.prm = prm;
      J.learned_wins = keep;
      J.rho_learned = rho;
      J.rho_classical = rho_c;
      J.krylov_learned = kl;
      J.krylov_classical = kc;
    }
  } else if (!keep) {
    H.L.resize(1);
    build_levels(c, cl, info);
  }
  report(rho, rho_c, kl, kc, keep);
}

void amg_setup_level0(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info) {
  c->keep_valid = false;
  if (prm.coupled) {
    vanka_setup(c, prm, info);
    return;
  }
  c->precond_kind = 0;
  Hierarchy& H = c->H;
  HIP_CHECK(hipEventRecord(c->ev0, c->stream));  // set-up time includes the judge
  H.L.clear();
  H.L.emplace_back();
  Level& L0 = H.L[0];
  copy_csr(c, c->A, L0.A);
  L0.n = c->A.rows;
  L0.comp.ensure(L0.n);
  k_comp_mod3<<<div_up(L0.n, 256), 256, 0, c->stream>>>(L0.n, L0.comp.p);
  HIP_LAUNCH_CHECK();
  // 3x3 node-block copy of A (entries removed from the CSR by the Dirichlet
  // elimination are exact zeros in the eliminated tangent)
  L0.bptr = c->nptr.p;
  L0.bcol = c->ncol.p;
  L0.nbr = c->n;
  L0.b3d.ensure(9 * (size_t)c->nb);
  L0.b3f.ensure(9 * (size_t)c->nb);
  k_block3<<<div_up(9L * c->nb, 256), 256, 0, c->stream>>>(c->nb, c->Kval.p, L0.b3d.p, L0.b3f.p);
  HIP_LAUNCH_CHECK();
  build_hierarchy(c, prm, info);
  H.reusable = true;
  HIP_CHECK(hipEventRecord(c->ev1, c->stream));
  if (info) info->seconds = elapsed_ms(c) * 1e-3;
}

// Re-set-up on the coarse grids of the last set-up of this mesh's tangent:
// the splittings, P and R (and the learned level-0 rows, if kept) stay; level
// 0 takes the displacement block of the last assembly, every coarser operator
// is again the Galerkin product R A P, and the smoother data, coarsest inverse
// and cycle copies are rebuilt.  No strength, PMIS, interpolation or judge.
void amg_resetup_level0(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info) {
  c->keep_valid = false;
  if (prm.coupled) {  // the coupled hierarchy is always built anew
    vanka_setup(c, prm, info);
    return;
  }
  c->precond_kind = 0;
  Hierarchy& H = c->H;
  hipStream_t s = c->stream;
  if (!H.reusable || H.L.empty() || H.L[0].n != c->A.rows || H.L[0].A.nnz != c->A.nnz)
    fail(HFSI_E_ORDER, "amg_resetup: no hierarchy of this mesh's tangent to reuse");
  HIP_CHECK(hipEventRecord(c->ev0, s));
  const int prev_precision = H.precision;
  H.ready = false;
  H.reusable = false;
  set_schedule(H, prm);
  AuxJoin aux_join{c};
  H.lmax_dev.ensure(32);
  H.setup_flags.zero(1, s);
  Level& L0 = H.L[0];
  HIP_CHECK(hipMemcpyAsync(L0.A.val.p, c->A.val.p, sizeof(double) * c->A.nnz, hipMemcpyDeviceToDevice, s));
  k_block3<<<div_up(9L * c->nb, 256), 256, 0, s>>>(c->nb, c->Kval.p, L0.b3d.p, L0.b3f.p);
  HIP_LAUNCH_CHECK();
  const int nl = (int)H.L.size();
  for (int l = 0; l < nl; ++l) {
    smoother_data(c, H.L[l], prm, l);
    if (l + 1 == nl) break;
    Level& Lf = H.L[l];
    spgemm_values(c, Lf.A, Lf.P, Lf.AP, Lf.p_rowmax, H.setup_flags.p);
    spgemm_values(c, Lf.R, Lf.AP, H.L[l + 1].A, Lf.ap_rowmax, H.setup_flags.p, !(H.drop_tol > 0.0));
    if (prm.precision == 1 && prev_precision != 1) to_f32_transfer(c, Lf);  // P, R unchanged
  }
  finish_hierarchy(c, prm, true);
  H.reusable = true;
  fill_info(H, info, 0, -1.0);
  HIP_CHECK(hipEventRecord(c->ev1, s));
  if (info) info->seconds = elapsed_ms(c) * 1e-3;
}

void check_amg_params(const hfsi_amg_params* p) {
  if (!p || p->struct_size != sizeof(hfsi_amg_params)) fail(HFSI_E_ARG, "amg params: struct_size mismatch");
  if (!(p->strength_theta > 0.0 && p->strength_theta <= 1.0)) fail(HFSI_E_ARG, "amg params: theta in (0,1]");
  if (p->max_coarse < 1 || p->max_levels < 1) fail(HFSI_E_ARG, "amg params: bad level limits");
  if (p->smoother < 0 || p->smoother > 1 || p->nu_pre < 0 || p->nu_post < 0 || p->nu_pre_coarse < 0 ||
      p->nu_post_coarse < 0 || p->nu_pre + p->nu_post < 1 || p->nu_pre_coarse + p->nu_post_coarse < 1)
    fail(HFSI_E_ARG, "amg params: bad smoother or sweep counts");
  if (p->precision < 0 || p->precision > 1) fail(HFSI_E_ARG, "amg params: bad precision");
  for (int d : {p->cheb_degree, p->cheb_degree_pre, p->cheb_degree_coarse})
    if (d < 1 || d > 8) fail(HFSI_E_ARG, "amg params: Chebyshev degrees in 1..8");
  if (!(p->cheb_ratio > 1.0)) fail(HFSI_E_ARG, "amg params: Chebyshev ratio > 1");
  if (p->interp_kind < 0 || p->interp_kind > 1 || p->p_max < 0)
    fail(HFSI_E_ARG, "amg params: interp_kind 0 or 1, p_max >= 0");
  if (p->interp < 0 || p->interp > 1) fail(HFSI_E_ARG, "amg params: interp must be 0 (classical) or 1 (learned)");
  if (p->judge_classical < 0 || p->judge_classical > 2) fail(HFSI_E_ARG, "amg params: judge_classical in 0..2");
  if (!(p->drop_tol >= 0.0 && p->drop_tol < 1.0)) fail(HFSI_E_ARG, "amg params: drop_tol in [0, 1)");
  if (p->coupled < 0 || p->coupled > 2) fail(HFSI_E_ARG, "amg params: coupled in 0..2");
  if (p->coupled) {
    if (!(p->vanka_omega > 0.0 && p->vanka_omega < 2.0) || p->vanka_steps < 0 || p->vanka_steps > 64)
      fail(HFSI_E_ARG, "amg params: vanka_omega in (0, 2), vanka_steps in 0..64");
    if (p->interp != 0 || p->drop_tol != 0.0)
      fail(HFSI_E_ARG, "amg params: the coupled hierarchy takes interp 0 and drop_tol 0");
  }
}

bool same_amg_params(const hfsi_amg_params& a, const hfsi_amg_params& b) {
  return a.strength_theta == b.strength_theta && a.max_coarse == b.max_coarse && a.max_levels == b.max_levels &&
         a.seed == b.seed && a.smoother == b.smoother && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post &&
         a.precision == b.precision && a.interp == b.interp && a.fallback_rho == b.fallback_rho &&
         a.cheb_degree == b.cheb_degree && a.cheb_ratio == b.cheb_ratio && a.interp_kind == b.interp_kind &&
         a.p_max == b.p_max && a.cheb_degree_pre == b.cheb_degree_pre && a.nu_post_coarse == b.nu_post_coarse &&
         a.cheb_degree_coarse == b.cheb_degree_coarse && a.nu_pre_coarse == b.nu_pre_coarse &&
         a.judge_classical == b.judge_classical && a.drop_tol == b.drop_tol && a.coupled == b.coupled &&
         a.vanka_omega == b.vanka_omega && a.vanka_steps == b.vanka_steps;
}

}  // namespace hfsi

extern "C" hfsi_status hfsi_amg_setup(hfsi_ctx* c, const hfsi_amg_params* prm, hfsi_amg_info* info) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 4, "amg_setup");
  hfsi::check_amg_params(prm);
  if (info && info->struct_size != sizeof(hfsi_amg_info)) fail(HFSI_E_ARG, "amg info: struct_size mismatch");
  hfsi::amg_setup_level0(c, *prm, info);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_amg_resetup(hfsi_ctx* c, const hfsi_amg_params* prm, hfsi_amg_info* info) {
  HFSI_ABI_BEGIN(c)
  require_stage(c, 4, "amg_resetup");
  hfsi::check_amg_params(prm);
  if (info && info->struct_size != sizeof(hfsi_amg_info)) fail(HFSI_E_ARG, "amg info: struct_size mismatch");
  hfsi::amg_resetup_level0(c, *prm, info);
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_amg_setup_csr(hfsi_ctx* c, int32_t n, const int32_t* ptr, const int32_t* col,
                                          const double* val, const int32_t* comp, const hfsi_amg_params* prm,
                                          hfsi_amg_info* info) {
  HFSI_ABI_BEGIN(c)
  hfsi::check_amg_params(prm);
  if (n <= 0 || !ptr || !col || !val || !comp) fail(HFSI_E_ARG, "amg_setup_csr: bad arguments");
  if (prm->coupled) fail(HFSI_E_ARG, "amg_setup_csr: the coupled hierarchy needs the assembled tangent");
  if (info && info->struct_size != sizeof(hfsi_amg_info)) fail(HFSI_E_ARG, "amg info: struct_size mismatch");
  c->keep_valid = false;
  const int64_t nnz = ptr[n];
  if (ptr[0] != 0 || nnz < n) fail(HFSI_E_ARG, "amg_setup_csr: bad row pointer");
  for (int i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) fail(HFSI_E_ARG, "amg_setup_csr: row pointer not monotone");
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) fail(HFSI_E_ARG, "amg_setup_csr: column out of range");
      if (e > ptr[i] && col[e] <= col[e - 1]) fail(HFSI_E_ARG, "amg_setup_csr: columns not strictly ascending");
    }
  }
  c->precond_kind = 0;
  hfsi::Hierarchy& H = c->H;
  H.L.clear();
  H.L.emplace_back();
  hfsi::Level& L0 = H.L[0];
  L0.n = n;
  L0.A.rows = L0.A.cols = n;
  L0.A.nnz = nnz;
  L0.A.ptr.upload(ptr, n + 1, c->stream);
  L0.A.col.upload(col, nnz, c->stream);
  L0.A.val.upload(val, nnz, c->stream);
  L0.comp.upload(comp, n, c->stream);
  HIP_CHECK(hipEventRecord(c->ev0, c->stream));  // device set-up after the uploads
  hfsi::build_hierarchy(c, *prm, info);
  HIP_CHECK(hipEventRecord(c->ev1, c->stream));
  if (info) info->seconds = hfsi::elapsed_ms(c) * 1e-3;
  HFSI_ABI_END(c)
}

extern "C" hfsi_status hfsi_amg_export(hfsi_ctx* c, int32_t level, int32_t which, int32_t* rows, int32_t* cols,
                                       int64_t* nnz, int32_t* ptr, int32_t* col, double* val, uint8_t* val_u8) {
  HFSI_ABI_BEGIN(c)
  if (which >= 10) {
    hfsi::vanka_export(c, level, which, rows, cols, nnz, ptr, col, val);
    return HFSI_OK;
  }
  hfsi::Hierarchy& H = c->H;
  if (!H.ready) fail(HFSI_E_ORDER, "amg_export: no hierarchy");
  if (level < 0 || level >= (int)H.L.size()) fail(HFSI_E_ARG, "amg_export: level out of range");
  hfsi::Level& L = H.L[level];
  const bool last = level == (int)H.L.size() - 1;
  hipStream_t s = c->stream;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  };
  if (which == 0 || which == 1) {
    if (which == 1 && last) fail(HFSI_E_ARG, "amg_export: the coarsest level has no P");
    const hfsi::Csr<double>& M = which == 0 ? L.A : L.P;
    if (rows) *rows = M.rows;
    if (cols) *cols = M.cols;
    if (nnz) *nnz = M.nnz;
    cp(ptr, M.ptr.p, sizeof(int) * (M.rows + 1));
    cp(col, M.col.p, sizeof(int) * M.nnz);
    cp(val, M.val.p, sizeof(double) * M.nnz);
  } else if (which == 2 || which == 3) {
    if (last) fail(HFSI_E_ARG, "amg_export: the coarsest level has no splitting");
    if (rows) *rows = L.n;
    if (cols) *cols = 0;
    const int64_t k = which == 2 ? L.A.nnz : L.n;
    if (nnz) *nnz = k;
    cp(val_u8, which == 2 ? (const void*)L.strong.p : (const void*)L.state.p, (size_t)k);
  } else if (which == 4) {
    if (rows) *rows = L.n;
    if (cols) *cols = 0;
    if (nnz) *nnz = L.n;
    cp(col, L.comp.p, sizeof(int) * L.n);
  } else {
    fail(HFSI_E_ARG, "amg_export: unknown item");
  }
  HIP_CHECK(hipStreamSynchronize(s));
  HFSI_ABI_END(c)
}
