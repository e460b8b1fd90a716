/* A C program that uses the library through its C ABI only: it reads a
 * problem (mesh, materials, boundary data) from a binary file, applies the
 * load in increments with Newton's method (hfsi_newton_solve, Section
 * "Newton's Method") and writes the final state.
 *
 *   newton_driver <problem file> <increments> <state out> [adaptive 0/1] [weights | coupled | additive]
 *
 * Problem file, little endian: int64 n, m, k; double X[n][3]; int32
 * tets[m][4]; int32 mat_id[m]; uint8 dir_mask[n][4]; int32 tris[k][3];
 * double traction[k][3]; int32 n_mat; per material int32 model and double
 * c10, c01, kappa, k1, k2; optionally int32 has_lattice and, if it is 1,
 * int32 lattice[n][3] (the integer lattice coordinates the learned
 * interpolation needs).  With a weight file (hfsi_mlp_load format) the
 * level-0 interpolation is the learned one under the classical judge and the
 * V-cycle runs in fp32; with the word "coupled" the linear systems are
 * preconditioned by the coupled displacement-pressure AMG with the
 * multiplicative Vanka smoother (omega 0.78, 6 sweeps; section "The
 * multiplicative Vanka smoother"), with "additive" by the same hierarchy
 * with the additive Vanka variant (omega 0.8, 6 sweeps); otherwise classical
 * interpolation and an fp64 cycle.
 * State out: double v[n][4].  Exit status 0 when every increment converged. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hfsi.h"

static int read_all(FILE* f, void* p, size_t size, size_t cnt) { return fread(p, size, cnt, f) == cnt; }

static void* take(size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of host memory\n");
    exit(2);
  }
  return p;
}

/* defaults documented in hfsi.h */
static hfsi_newton_solve_params default_params(int adaptive, int learned, int coupled) {
  hfsi_newton_solve_params p;
  memset(&p, 0, sizeof p);  /* every field not set below is zero */
  hfsi_amg_params* a = &p.step.amg;
  hfsi_solve_params* s = &p.step.solve;
  p.struct_size = sizeof p;
  p.step.struct_size = sizeof p.step;
  p.step.amg_reuse = 0;
  a->struct_size = sizeof *a;
  a->strength_theta = 0.15;
  a->max_coarse = 500;
  a->max_levels = 25;
  a->seed = 12345;
  a->smoother = 1;
  a->nu_pre = 1;
  a->nu_post = 1;
  a->precision = learned ? 1 : 0;
  a->interp = learned ? 1 : 0;
  a->fallback_rho = 0.5;
  a->cheb_degree = 3;
  a->cheb_ratio = 30.0;
  a->interp_kind = 1;
  a->p_max = 4;
  a->cheb_degree_pre = 1;
  a->nu_post_coarse = 1;
  a->cheb_degree_coarse = 3;
  a->nu_pre_coarse = 0;
  a->judge_classical = 2;
  a->drop_tol = 0.0;
  a->coupled = coupled;
  a->vanka_omega = coupled == 2 ? 0.8 : 0.78;
  a->vanka_steps = 6;
  s->struct_size = sizeof *s;
  s->tol = 1e-8;
  s->restart = 50;
  s->max_iter = 500;
  s->method = 0;
  s->precond_form = 0;
  p.eps2 = 1e-10;
  p.max_newton = 25;
  p.adaptive = adaptive;
  p.eps1_max = 1e-2;
  p.eps1_min = 1e-12;
  p.line_search = 0;
  p.ref_norm = 0.0;
  return p;
}

#define CHECK(call)                                                                        \
  do {                                                                                     \
    hfsi_status st_ = (call);                                                              \
    if (st_ != HFSI_OK) {                                                                  \
      fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, hfsi_last_error(ctx));      \
      return 1;                                                                            \
    }                                                                                      \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: %s <problem file> <increments> <state out> [adaptive] [weights | coupled | additive]\n", argv[0]);
    return 2;
  }
  const int increments = atoi(argv[2]);
  const int adaptive = argc > 4 ? atoi(argv[4]) : 0;
  const int coupled = argc <= 5 ? 0 : strcmp(argv[5], "coupled") == 0 ? 1 : strcmp(argv[5], "additive") == 0 ? 2 : 0;
  const char* weights = argc > 5 && !coupled ? argv[5] : NULL;
  FILE* f = fopen(argv[1], "rb");
  if (!f || increments < 1) {
    fprintf(stderr, "cannot read %s or bad increment count\n", argv[1]);
    return 2;
  }
  int64_t n = 0, m = 0, k = 0;
  int ok = read_all(f, &n, 8, 1) && read_all(f, &m, 8, 1) && read_all(f, &k, 8, 1);
  if (!ok || n <= 0 || m <= 0 || k < 0) {
    fprintf(stderr, "bad header\n");
    return 2;
  }
  double* X = take(sizeof(double) * 3 * n);
  int32_t* tets = take(sizeof(int32_t) * 4 * m);
  int32_t* mat = take(sizeof(int32_t) * m);
  uint8_t* dir = take(4 * n);
  int32_t* tris = take(sizeof(int32_t) * 3 * k);
  double* trac = take(sizeof(double) * 3 * k);
  ok = read_all(f, X, 8, 3 * n) && read_all(f, tets, 4, 4 * m) && read_all(f, mat, 4, m) &&
       read_all(f, dir, 1, 4 * n) && read_all(f, tris, 4, 3 * k) && read_all(f, trac, 8, 3 * k);
  int32_t n_mat = 0;
  ok = ok && read_all(f, &n_mat, 4, 1) && n_mat > 0 && n_mat < 64;
  if (!ok) {
    fprintf(stderr, "truncated problem file\n");
    return 2;
  }
  hfsi_material* mats = take(sizeof(hfsi_material) * n_mat);
  for (int i = 0; i < n_mat; ++i) {
    double c[5];
    if (!read_all(f, &mats[i].model, 4, 1) || !read_all(f, c, 8, 5)) {
      fprintf(stderr, "truncated material table\n");
      return 2;
    }
    mats[i].struct_size = sizeof(hfsi_material);
    mats[i].c10 = c[0];
    mats[i].c01 = c[1];
    mats[i].kappa = c[2];
    mats[i].k1 = c[3];
    mats[i].k2 = c[4];
    mats[i].theta = 0.0;
  }
  int32_t has_lattice = 0;
  int32_t* lattice = NULL;
  if (read_all(f, &has_lattice, 4, 1) && has_lattice == 1) {
    lattice = take(sizeof(int32_t) * 3 * n);
    if (!read_all(f, lattice, 4, 3 * n)) {
      fprintf(stderr, "truncated lattice coordinates\n");
      return 2;
    }
  }
  fclose(f);
  if (weights && !lattice) {
    fprintf(stderr, "the learned interpolation needs lattice coordinates in the problem file\n");
    return 2;
  }

  hfsi_ctx* ctx = NULL;
  if (hfsi_create(&ctx, 0, NULL) != HFSI_OK) {
    fprintf(stderr, "hfsi_create failed\n");
    return 1;
  }
  CHECK(hfsi_set_mesh(ctx, n, X, m, tets, mat, lattice, NULL));
  CHECK(hfsi_set_materials(ctx, n_mat, mats));
  CHECK(hfsi_set_bc(ctx, dir, k, tris, trac));
  double* v = NULL;
  if (hipMalloc((void**)&v, sizeof(double) * 4 * n) != hipSuccess || hipMemset(v, 0, sizeof(double) * 4 * n) != hipSuccess) {
    fprintf(stderr, "device allocation failed\n");
    return 1;
  }
  if (weights) CHECK(hfsi_mlp_load(ctx, weights));
  const hfsi_newton_solve_params prm = default_params(adaptive, weights != NULL, coupled);
  int all = 1;
  for (int inc = 1; inc <= increments; ++inc) {
    hfsi_newton_solve_info info;
    info.struct_size = sizeof info;
    const hfsi_status st = hfsi_newton_solve(ctx, v, (double)inc / increments, &prm, &info);
    if (st < 0) {
      fprintf(stderr, "hfsi_newton_solve failed (%d): %s\n", (int)st, hfsi_last_error(ctx));
      return 1;
    }
    printf("increment %d: %d Newton, %d Krylov iterations, converged %d\n", inc, info.newton_iterations,
           info.krylov_iterations, info.converged);
    all = all && info.converged;
  }
  double* h = take(sizeof(double) * 4 * n);
  if (hipMemcpy(h, v, sizeof(double) * 4 * n, hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "copy failed\n");
    return 1;
  }
  FILE* o = fopen(argv[3], "wb");
  if (!o || fwrite(h, 8, 4 * n, o) != (size_t)(4 * n)) {
    fprintf(stderr, "cannot write %s\n", argv[3]);
    return 1;
  }
  fclose(o);
  (void)hipFree(v);
  (void)hfsi_destroy(ctx);
  free(X); free(tets); free(mat); free(dir); free(tris); free(trac); free(mats); free(h); free(lattice);
  return all ? 0 : 3;
}
