// Shared internals of the hfsi HIP library: error handling, device buffers,
// the context object and small device utilities (scan, reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "hfsi.h"

namespace hfsi {

// Every internal failure is thrown as Error and turned into a status code at
// the ABI boundary (see HFSI_ABI_BEGIN / HFSI_ABI_END).
struct Error : std::runtime_error {
  hfsi_status code;
  Error(hfsi_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(hfsi_status c, const std::string& m) { throw Error(c, m); }

#define HIP_CHECK(expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::hfsi::fail(e_ == hipErrorOutOfMemory ? HFSI_E_OOM : HFSI_E_HIP,                     \
                   std::string(#expr) + ": " + hipGetErrorString(e_) + " at " + __FILE__ + \
                       ":" + std::to_string(__LINE__));                                     \
  } while (0)

#define HIP_LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// Device memory comes from a per-process block cache.  A block released by a
// DevBuf returns to the cache tagged with the stream of the library call that
// released it (every kernel of a context runs on that context's stream) and
// is handed out again only for work on the same stream, so stream order makes
// the reuse safe; blocks released after a stream synchronisation (context
// destruction) are free for any stream.  hipMalloc runs only when no cached
// block of 1x..2x the request fits; no hipFree (which synchronises the
// device) runs while a context is alive.
extern thread_local hipStream_t tls_stream;  // stream of the current library call
extern thread_local bool tls_idle;           // releases happen after a stream sync

// Tags the device blocks released in its scope with another stream (declare
// it before the buffers it covers).
struct StreamTag {
  hipStream_t saved;
  explicit StreamTag(hipStream_t s) : saved(tls_stream) { tls_stream = s; }
  ~StreamTag() { tls_stream = saved; }
  StreamTag(const StreamTag&) = delete;
  StreamTag& operator=(const StreamTag&) = delete;
};
void* dev_alloc(size_t bytes, size_t* cap, int* dev);
void dev_release(void* p, size_t cap, int dev);
void dev_cache_trim();  // hipFree every idle cached block (no context alive)

// Device buffer owned by the context or by one library call.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;    // elements the block holds
  size_t cap = 0;  // bytes of the block
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap), dev(o.dev) {
    o.p = nullptr;
    o.n = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      dev = o.dev;
      o.p = nullptr;
      o.n = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) dev_release(p, cap, dev);
    p = nullptr;
    n = cap = 0;
  }
  // (re)allocate to at least cnt elements; contents are not preserved
  void ensure(size_t cnt) {
    if (cnt <= n && p) return;
    release();
    p = (T*)dev_alloc((cnt ? cnt : 1) * sizeof(T), &cap, &dev);
    n = cap / sizeof(T);
  }
  void upload(const T* h, size_t cnt, hipStream_t s) {
    ensure(cnt);
    if (cnt) HIP_CHECK(hipMemcpyAsync(p, h, cnt * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void zero(size_t cnt, hipStream_t s) {
    ensure(cnt);
    if (cnt) HIP_CHECK(hipMemsetAsync(p, 0, cnt * sizeof(T), s));
  }
  std::vector<T> download(size_t cnt, hipStream_t s) const {
    std::vector<T> h(cnt);
    if (cnt) {
      HIP_CHECK(hipMemcpyAsync(h.data(), p, cnt * sizeof(T), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
    }
    return h;
  }
};

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Output k of the SplitMix64 stream seeded with `seed` (Steele, Lea & Flood,
// OOPSLA 2014): mix(seed + (k + 1) * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Lanes per row of the padded CSR layout: 3 to 6 chunks per lane (8 lanes
// for the 25-35 chunks of the first coarse levels measured fastest), more
// lanes on small levels so that the launch still spreads over the whole chip.
// Lane g of a row takes the row's chunks g, g+G, g+2G, ...; within a group of
// q <= G consecutive chunks starting at entry e0, slot t of chunk g holds
// entry e0 + g + q t, so that the G lanes' t-th gathers read G consecutive
// (sorted) columns.
inline int lanes_for4(int64_t chunks, int rows) {
  const double avg = rows ? (double)chunks / rows : 1.0;
  int G = 2;
  while (G < 64 && 6.0 * G <= avg) G *= 2;
  while (G < 64 && (int64_t)rows * G < 65536) G *= 2;
  return G;
}

// --------------------------------------------------------------- CSR matrix
template <class V>
struct Csr {
  int rows = 0, cols = 0;
  int64_t nnz = 0;
  DevBuf<int> ptr, col;
  DevBuf<V> val;
};

// CSR copy for the smoother and residual of levels without node blocks: each
// row padded to a multiple of 4 entries (zero values, column offset 0), so a
// lane reads 4 values and 4 columns with one aligned load each.  Columns are
// 16-bit offsets from the row's smallest column (`base`); a row that spans
// more than 65535 columns (a few rows of the large coarse levels) keeps
// absolute int32 columns in a side array instead: its base is -1 - w, w its
// index among those rows, and its chunk k sits at chunk k + wch[w] of c32w.
struct Packed4 {
  int rows = 0;
  int64_t chunks = 0;          // padded entries / 4
  int nwide = 0;               // rows with int32 columns
  int64_t wchunks = 0;         // their chunks
  DevBuf<int> p4;              // [rows+1] first chunk of each row
  DevBuf<int> base;            // [rows] smallest column, or -1 - w
  DevBuf<uint16_t> c16;        // [4*chunks] column - base (narrow rows)
  DevBuf<int> c32w;            // [4*wchunks] columns of the wide rows
  DevBuf<int> wch;             // [nwide] chunk shift of each wide row
  DevBuf<float> v32;           // [4*chunks] values of the fp32 cycle
  DevBuf<double> v64;          // [4*chunks] values of the fp64 cycle
};

// ------------------------------------------------------------- AMG level
struct Level {
  int n = 0;
  Csr<double> A;           // fp64 operator
  DevBuf<float> A32;       // fp32 copy of A.val (mixed precision)
  DevBuf<int> comp;        // unknown component of each row
  DevBuf<uint8_t> strong;  // strength flag per A entry
  DevBuf<int8_t> state;    // +1 C, -1 F
  DevBuf<int> cidx;        // coarse index of C points (exclusive scan)
  Csr<double> P, R;        // interpolation and restriction (R = P^T)
  DevBuf<float> P32, R32;
  Csr<double> AP;          // A P, kept for a re-set-up on the same pattern
  int p_rowmax = 0;        // longest row of P, and of AP
  int ap_rowmax = 0;
  DevBuf<double> dinv;     // smoother diagonal (l1 or plain), fp64
  DevBuf<float> dinv32;
  double lmax = 0.0;       // Chebyshev upper eigenvalue estimate
  // level 0 built from the assembled tangent: the same operator as 3x3 node
  // blocks (one column index per 9 values) for the smoother and residual
  const int* bptr = nullptr;  // node-block row pointer (context-owned)
  const int* bcol = nullptr;
  int nbr = 0;                // node rows
  DevBuf<double> b3d;         // [9 * blocks]
  DevBuf<float> b3f;
  // other levels: padded copy of A in the cycle's precision
  bool packed = false;
  Packed4 pk;
  // V-cycle vectors (fp64 and fp32 variants used according to precision)
  DevBuf<double> x, b, r, t;
  DevBuf<float> xf, bf, rf, tf;
};

struct Hierarchy {
  std::vector<Level> L;
  int nc = 0;                 // coarsest size
  // the coarsening stalled (a level would keep more than 90% of its rows);
  // above the dense limit the coarsest level is then solved by
  // kCoarseSweeps l1-Jacobi sweeps from zero instead of its inverse
  bool stalled = false;
  bool coarse_iterative = false;
  DevBuf<double> coarse_inv;  // explicit inverse of the coarsest operator
  DevBuf<double> lmax_dev;    // per-level eigenvalue estimates (written on the aux stream)
  DevBuf<int> setup_flags;    // numeric sparse-product overflow, read with the estimates
  int precision = 0;
  int smoother = 0;
  int nu_pre = 1, nu_post = 1;  // level 0: sweeps before / after the correction
  int nu_pre_coarse = 0, nu_post_coarse = 1;  // the same on levels >= 1
  int cheb_degree = 3;          // Chebyshev degrees: level-0 post, pre, coarse post
  int cheb_degree_pre = 1, cheb_degree_coarse = 3;
  double cheb_ratio = 30.0;     // interval [lmax / ratio, 1.1 lmax]
  bool ready = false;
  int learned = 0;        // 1 if level 0 carries the learned interpolation
  double drop_tol = 0.0;  // coarse-operator sparsification of the set-up (a
                          // re-set-up keeps the sparsified patterns)
  bool reusable = false;  // built from this mesh's assembled tangent: its
                          // coarse grids may be kept by a re-set-up
};

}  // namespace hfsi

constexpr int kMaxDenseCoarse = 4096;  // rows of the coarsest level inverted densely
constexpr int kCoarseSweeps = 16;      // l1-Jacobi sweeps on a larger coarsest level

// ------------------------------------------------------------- the context
struct hfsi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int stage = 0;  // 0 created, 1 mesh, 2 materials, 3 bc, 4 assembled, 5 amg ready

  // mesh (elements stored in colour order; perm[k] = original element index)
  int n = 0, m = 0;
  hfsi::DevBuf<double> X;      // [n*3]
  hfsi::DevBuf<int> tets;      // [4*m] SoA: tets[a*m + e]
  hfsi::DevBuf<int> mat;       // [m]
  hfsi::DevBuf<double> G;      // [12*m] SoA: G[(a*3+J)*m + e]
  hfsi::DevBuf<double> V, h;   // [m]
  hfsi::DevBuf<double> fib;    // [6*m] SoA or empty
  hfsi::DevBuf<int> lattice;   // [3*n] or empty
  bool has_fib = false, has_lattice = false;
  std::vector<int> perm;       // colour order -> original element
  std::vector<int> colour_ptr; // element ranges per colour
  // node-block pattern
  int nb = 0;
  hfsi::DevBuf<int> nptr, ncol;  // [n+1], [nb]
  hfsi::DevBuf<int> slot;        // [16*m] SoA: slot[(a*4+b)*m + e]
  hfsi::DevBuf<int> diag_blk;    // [n]
  hfsi::DevBuf<int> brow;        // [nb] block row of each block
  hfsi::DevBuf<double> Kval;     // [16*nb]
  hfsi::DevBuf<double> Mval;     // [nb] scalar P1 mass on the node pattern
  hfsi::DevBuf<double> b2;       // [3*nb] pressure row (B2 part) of every block
  // materials
  int n_mat = 0;
  hfsi::DevBuf<double> mtab;     // [n_mat * 8]: model,c10,c01,kappa,k1,k2,mu_l,theta
  std::vector<double> mtab_h;
  // boundary
  hfsi::DevBuf<uint8_t> dir;     // [4n]
  hfsi::DevBuf<double> fext;     // [3n] nodal load at load factor 1
  // Newmark-beta inertia: cm = rho_s / (beta dt^2) (0 = quasi-static) and
  // the history field r_s [3n] of the current time step
  double nm_rho = 0.0, nm_beta = 0.625, nm_gamma = 1.0, nm_dt = 0.0, cm = 0.0;
  hfsi::DevBuf<double> rs;
  hfsi::DevBuf<double> schur;    // [n]
  // A block (scalar CSR over 3n dofs) and its source positions in Kval
  hfsi::Csr<double> A;
  hfsi::DevBuf<int> a_src;
  // hierarchy
  hfsi::Hierarchy H;
  // verdict of the classical judge of the learned interpolation, kept for
  // the later set-ups of the same problem, weights and parameters (reset by
  // set_mesh, set_materials, set_bc and any change of the weights)
  struct {
    bool valid = false;
    bool learned_wins = false;
    double rho_learned = -1.0, rho_classical = -1.0;
    double krylov_learned = -1.0, krylov_classical = -1.0;
    hfsi_amg_params prm{};
  } judge;
  // Krylov workspace
  hfsi::DevBuf<double> kv;       // basis V [(m+1) * N]
  hfsi::DevBuf<double> kz;       // Z [m * N]
  hfsi::DevBuf<double> kw, kr, ktmp, kdv;
  hfsi::DevBuf<double> kvprev;  // state at the start of a time step
  hfsi::DevBuf<double> ktrial, ktres;  // damped Newton: trial state and its residual
  hfsi::DevBuf<double> kred;     // reduction partials
  hfsi::DevBuf<double> kh;       // Hessenberg / Givens state on device
  double* pinned = nullptr;      // host-pinned scalars
  hfsi::DevBuf<double> scal;     // device scalars
  hfsi::DevBuf<int> iscal;       // device integer scalars
  void* mlp_impl = nullptr;      // learned-interpolation state (mlp.hip)
  void* vanka_impl = nullptr;    // coupled (u,p) AMG with the Vanka smoother (vanka.hip)
  void* fluid_impl = nullptr;    // fluid or mesh-Laplacian physics (fluid.hip); null: the structure
  int precond_kind = 0;          // preconditioner of the last set-up: 0 P_L, 1 coupled V-cycle
  int precond_form = 0;          // block form during a Krylov solve: 0 P_L, 1 P_R
  // Newton with amg_reuse = 3: the preconditioner of the last set-up made by
  // a Newton iteration on this context is kept whole while it stays usable
  bool keep_valid = false;       // such a preconditioner exists (any set-up or change of the problem clears it)
  bool keep_stale = false;       // a solve with it converged at under half its first rate: build anew
  hfsi_amg_params keep_prm{};    // the parameters of that set-up
  int keep_levels = 0;
  double keep_rate0 = 0.0;       // log10 residual reduction per iteration of its first solve (0: none yet)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t kev[2] = {nullptr, nullptr};  // FGMRES scalar read-back slots
  hipStream_t aux = nullptr;               // AMG set-up work off the critical path
  hipEvent_t aev[2] = {nullptr, nullptr};  // aux fork and join
};

namespace hfsi {

// ------------------------------------------------------------------ scans
// Exclusive prefix sum of `n` int32 values; out may alias in.  Returns the
// total (one wait on the stream); `n_extra` (at most 8) device ints from
// `extra` are copied to `extra_host` in the same wait.
int64_t exclusive_scan(const int* in, int* out, int n, hipStream_t s, const int* extra = nullptr, int n_extra = 0,
                       int* extra_host = nullptr);
// Same without reading back the total.
void exclusive_scan_async(const int* in, int* out, int n, hipStream_t s);

// Sum of a device double array (synchronises).
double device_sum(hfsi_ctx* c, const double* x, int n);

// Elapsed milliseconds between two events recorded on the context stream.
float elapsed_ms(hfsi_ctx* c);

void require_stage(hfsi_ctx* c, int st, const char* what);

// internal entry points implemented in the .hip files
void assemble(hfsi_ctx* c, const double* v, double load, double* R, hfsi_assembly_info* info);
void build_a_pattern(hfsi_ctx* c);
void amg_setup_level0(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info);
void amg_resetup_level0(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info);
void build_hierarchy(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info);
void check_amg_params(const hfsi_amg_params* p);
bool same_amg_params(const hfsi_amg_params& a, const hfsi_amg_params& b);
void vcycle_apply(hfsi_ctx* c, const double* r, double* z);
// z = P_L^{-1} r; with scale, the vector preconditioned is r / *scale, also
// written to rs
void precond_apply(hfsi_ctx* c, const double* r, double* z, const double* scale = nullptr, double* rs = nullptr);
void tangent_apply(hfsi_ctx* c, const double* x, double* y);
void fgmres_solve(hfsi_ctx* c, const double* b, double* x, const hfsi_solve_params& prm,
                  hfsi_solve_info* info);
// BiCGStab with the same preconditioner; krylov_solve picks by prm.method
void bicgstab_solve(hfsi_ctx* c, const double* b, double* x, const hfsi_solve_params& prm, hfsi_solve_info* info);
void krylov_solve(hfsi_ctx* c, const double* b, double* x, const hfsi_solve_params& prm, hfsi_solve_info* info);
double mass_norm(hfsi_ctx* c, const double* dv);
// coupled (u,p) AMG with the multiplicative Vanka smoother (vanka.hip)
void vanka_setup(hfsi_ctx* c, const hfsi_amg_params& prm, hfsi_amg_info* info);
void vanka_precond(hfsi_ctx* c, const double* r, double* z, const double* scale, double* rs);
void vanka_invalidate(hfsi_ctx* c);
void vanka_free(hfsi_ctx* c);
void vanka_export(hfsi_ctx* c, int level, int which, int32_t* rows, int32_t* cols, int64_t* nnz, int32_t* ptr,
                  int32_t* col, double* val);
// fluid and mesh-Laplacian contexts (fluid.hip): physics 0 structure, 1
// fluid, 2 mesh Laplacian
int physics_of(const hfsi_ctx* c);
void fluid_elements(hfsi_ctx* c, const double* v, double* R, bool want_K);
void fluid_schur(hfsi_ctx* c);
void fluid_free(hfsi_ctx* c);
// resolve the allocation-free entry point's scratch address on `device`
// (the current device); called once per context creation
void noalloc_scratch_init(int device);
// learned interpolation: correct level-0 P in place; free the state
void learned_correction(hfsi_ctx* c, Level& L);
void mlp_free(hfsi_ctx* c);
// rho = (||e_k||_A / ||e_0||_A)^{1/k} of k stationary V-cycles from a
// SplitMix64 start vector
double convergence_factor(hfsi_ctx* c, int cycles, uint64_t seed);
// (||r_k|| / ||r_0||)^(1/k) of k FGMRES steps on the assembled tangent with
// P_L on the current hierarchy, from a SplitMix64 right-hand side
double krylov_factor(hfsi_ctx* c, int k, uint64_t seed);
// minimum bytes one assembly must move; the element kernels alone (timing)
double assembly_bytes(hfsi_ctx* c);
void assemble_kernels_only(hfsi_ctx* c);

}  // namespace hfsi

#define HFSI_ABI_BEGIN(ctx)                     \
  if (!(ctx)) return HFSI_E_ARG;                \
  try {                                         \
    ::hfsi::tls_stream = (ctx)->stream;         \
    ::hfsi::tls_idle = false;                   \
    HIP_CHECK(hipSetDevice((ctx)->device));

#define HFSI_ABI_END(ctx)                       \
  }                                             \
  catch (const ::hfsi::Error& e) {              \
    (ctx)->err = e.what();                      \
    return e.code;                              \
  }                                             \
  catch (const std::exception& e) {             \
    (ctx)->err = e.what();                      \
    return HFSI_E_HIP;                          \
  }                                             \
  return HFSI_OK;
