/*
 * vlb_c_run.c -- a plain C caller of the library's C ABI (include/vlb.h):
 * one domain, stepped and read back, with no other runtime in the process.
 *
 *   vlb_c_run IN OUT NSTEPS
 *
 * IN holds a vlb_domain_desc, an int32 particle count n and n
 * vlb_particle_desc, as raw bytes in this ABI's layout.  The program
 * creates the domain on the default stream of device 0, sets the
 * particles, initialises, advances NSTEPS steps and writes to OUT the
 * fields rho, ux, uy, T, f_s and [df_s/dt] (nx*ny doubles each, row-major)
 * followed by the n vlb_particle_state records.  Exit status 0 on success;
 * otherwise the failing call and vlb_last_error() are printed.
 */
#include <stdio.h>
#include <stdlib.h>

#include "vlb.h"

static int fail(const char* what, vlb_status s, const vlb_ctx* c) {
  fprintf(stderr, "%s failed (%d): %s\n", what, (int)s, vlb_last_error(c));
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s IN OUT NSTEPS\n", argv[0]);
    return 2;
  }
  const long long nsteps = atoll(argv[3]);
  FILE* in = fopen(argv[1], "rb");
  if (!in) {
    perror(argv[1]);
    return 1;
  }
  vlb_domain_desc d;
  int32_t np = 0;
  if (fread(&d, sizeof d, 1, in) != 1 || fread(&np, sizeof np, 1, in) != 1 ||
      np < 0) {
    fprintf(stderr, "%s: short or bad input\n", argv[1]);
    return 1;
  }
  vlb_particle_desc* p = NULL;
  if (np > 0) {
    p = (vlb_particle_desc*)malloc((size_t)np * sizeof *p);
    if (!p || fread(p, sizeof *p, (size_t)np, in) != (size_t)np) {
      fprintf(stderr, "%s: short particle list\n", argv[1]);
      return 1;
    }
  }
  fclose(in);
  printf("vlb_c_run: library built from %s, %dx%d cells, %d particles, "
         "%lld steps\n", vlb_build_hash(), d.nx, d.ny, np, nsteps);
  fflush(stdout);

  vlb_ctx* c = NULL;
  vlb_status s = vlb_create(&d, NULL, &c);
  if (s != VLB_OK) return fail("vlb_create", s, NULL);
  if ((s = vlb_set_particles(c, np, p)) != VLB_OK)
    return fail("vlb_set_particles", s, c);
  if ((s = vlb_init(c)) != VLB_OK) return fail("vlb_init", s, c);
  if ((s = vlb_step(c, nsteps)) != VLB_OK) return fail("vlb_step", s, c);

  const size_t n = (size_t)d.nx * (size_t)d.ny;
  double* field = (double*)malloc(n * sizeof(double));
  vlb_particle_state* st =
      (vlb_particle_state*)malloc((size_t)(np > 0 ? np : 1) * sizeof *st);
  FILE* out = fopen(argv[2], "wb");
  if (!field || !st || !out) {
    fprintf(stderr, "cannot allocate or open %s\n", argv[2]);
    return 1;
  }
  const int32_t fields[6] = {VLB_FIELD_RHO, VLB_FIELD_UX, VLB_FIELD_UY,
                             VLB_FIELD_T, VLB_FIELD_FS, VLB_FIELD_DFS};
  for (int k = 0; k < 6; ++k) {
    if ((s = vlb_read_field(c, fields[k], field, 0)) != VLB_OK)
      return fail("vlb_read_field", s, c);
    if (fwrite(field, sizeof(double), n, out) != n) return 1;
  }
  if (np > 0) {
    if ((s = vlb_read_particles(c, np, st)) != VLB_OK)
      return fail("vlb_read_particles", s, c);
    if (fwrite(st, sizeof *st, (size_t)np, out) != (size_t)np) return 1;
  }
  fclose(out);
  vlb_destroy(c);
  free(field);
  free(st);
  free(p);
  printf("vlb_c_run: done\n");
  return 0;
}
