/* Host-side checks of libpe's host code, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: the offline
 * schedule builders over a grid of (l, T), the workspace layout and argument
 * validation over many shapes and option sets, tile-table parsing, and the
 * error paths of the online entry points that return before any device work.
 * No GPU is needed; exit status 0 when every expectation holds. */
#include <stdio.h>
#include <string.h>
#include <stdlib.h>
#include <math.h>
#include "pe.h"
int main(int argc, char** argv) {
  double abc[3 * 64], lu[2 * 65], err; int iters[64];
  int bad = 0;
  for (int T = 1; T <= 64; T *= 2)
    for (double ell = 1e-9; ell < 1.0; ell *= 7.3) {
      pe_status s = pe_coeffs(ell, T, NULL, abc, lu, &err, iters);
      if (s != PE_OK) { printf("coeffs %g %d -> %d\n", ell, T, s); bad++; }
      s = pe_coeffs_cubic(ell, T, NULL, abc, lu, &err);
      if (s != PE_OK) { printf("cubic %g %d -> %d\n", ell, T, s); bad++; }
    }
  /* invalid arguments */
  if (pe_coeffs(0.0, 5, NULL, abc, NULL, NULL, NULL) == PE_OK) bad++;
  if (pe_coeffs(1e-3, 0, NULL, abc, NULL, NULL, NULL) == PE_OK) bad++;
  if (pe_coeffs(1e-3, 65, NULL, abc, NULL, NULL, NULL) == PE_OK) bad++;
  if (pe_coeffs(1e-3, 5, NULL, NULL, NULL, NULL, NULL) == PE_OK) bad++;
  for (int st = 0; st < 8; ++st) if (!pe_status_string((pe_status)st)) bad++;
  /* workspace sizes over many shapes and options (host-only layout code) */
  pe_opts o; memset(&o, 0, sizeof o);
  o.T = 5; o.abc = abc; o.compute = PE_COMPUTE_BF16; o.force_class = -1;
  pe_coeffs(1e-3, 5, NULL, abc, NULL, NULL, NULL);
  pe_matrix mats[64]; memset(mats, 0, sizeof mats);
  static char dummy[16];
  for (int i = 0; i < 64; ++i) {
    mats[i].G = dummy; mats[i].X = dummy;
    mats[i].m = 1 + (i * 37) % 700; mats[i].n = 1 + (i * 91) % 1300;
    mats[i].ldg = mats[i].n; mats[i].ldx = mats[i].n;
    mats[i].g_dtype = PE_BF16; mats[i].x_dtype = PE_F32;
  }
  int computes[3] = {PE_COMPUTE_F32, PE_COMPUTE_BF16, PE_COMPUTE_FP8};
  for (int c = 0; c < 3; ++c)
    for (int tile = 0; tile <= 2; ++tile)
      for (int sk = 0; sk <= 4; sk += 4) {
        o.compute = computes[c]; o.tile = tile; o.split_k = sk;
        o.fp8_steps = computes[c] == PE_COMPUTE_FP8 ? 3 : 0;
        size_t b = pe_workspace_size(64, mats, &o);
        if (b == 0) { printf("ws 0 for compute %d tile %d\n", c, tile); bad++; }
        o.spectral_init = computes[c] != PE_COMPUTE_FP8 ? 8 : 0;
        b = pe_workspace_size(64, mats, &o);
        o.spectral_init = 0;
        if (computes[c] == PE_COMPUTE_F32 && tile != 2) { o.fast_restart = 3; o.fast_eps = 1e-3f;
          if (pe_workspace_size(64, mats, &o) == 0) bad++; o.fast_restart = 0; }
      }
  /* invalid shapes and options */
  o.compute = PE_COMPUTE_BF16; o.tile = 0; o.fp8_steps = 0;
  mats[3].ldg = 0;
  if (pe_workspace_size(64, mats, &o) != 0) bad++;
  mats[3].ldg = mats[3].n;
  o.T = 0; if (pe_workspace_size(64, mats, &o) != 0) bad++; o.T = 5;
  o.split_k = 65; if (pe_workspace_size(64, mats, &o) != 0) bad++; o.split_k = 0;
  if (pe_workspace_size(-1, mats, &o) != 0) bad++;
  /* tile table parsing */
  char tab[4096];
  snprintf(tab, sizeof tab, "%s/table.txt", argc > 1 ? argv[1] : ".");
  FILE* f = fopen(tab, "w");
  if (!f) { printf("cannot write %s\n", tab); return 1; }
  fprintf(f, "# c\nbf16_s1024_a1_xN 2\nbogus line\nf32_s256_a4_x1 1\n"); fclose(f);
  pe_tile_table_load(tab);
  pe_tile_table_load("/nonexistent/table");
  /* online entry points refuse a missing workspace before touching the device */
  o.compute = PE_COMPUTE_BF16; o.tile = 0;
  if (pe_polar(&mats[0], &o, NULL, 0, NULL) == PE_OK) bad++;
  if (pe_polar_batched(64, mats, &o, NULL, 0, NULL) == PE_OK) bad++;
  if (pe_polar(NULL, &o, NULL, 0, NULL) != PE_EINVAL) bad++;
  if (!pe_last_error()) bad++;
  if (pe_mlp_workspace_size(1000) == 0 || pe_mlp_workspace_size(0) != 0) bad++;
  printf("host checks: %d failures\n", bad);
  return bad != 0;
}
