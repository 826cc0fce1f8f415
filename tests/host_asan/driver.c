/* Host-side checks of libabcs under AddressSanitizer: every call here runs on
 * the host only (descriptor validation, layout, launch table, error strings),
 * or stops at the first device call when no device is present.  Exit status 0
 * when every check holds; AddressSanitizer aborts on a memory error. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "abcs.h"

static int failures = 0;
#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static abcs_image img(int h, int w, int B, double cr, int method) {
  abcs_image d;
  memset(&d, 0, sizeof d);
  d.height = h;
  d.width = w;
  d.row_pitch = (w + 3) / 4 * 4;
  d.block = B;
  d.subrate = cr;
  d.method = method;
  d.transform = ABCS_DCT;
  return d;
}

int main(void) {
  /* request sizes: every block size, rule and a range of shapes and rates */
  const int blocks[3] = {8, 16, 32};
  for (int bi = 0; bi < 3; ++bi)
    for (int m = 0; m < 3; ++m)
      for (int h = 1; h < 300; h += 37)
        for (int w = 1; w < 300; w += 41)
          for (int c = 1; c <= 10; ++c) {
            abcs_image d = img(h, w, blocks[bi], 0.05 * c, m);
            int64_t nb = -1, nm = -1, np = -1;
            const int st = abcs_image_totals(&d, &nb, &nm, &np);
            if (st == ABCS_OK) {
              const int B = blocks[bi];
              CHECK(nb == (int64_t)(h / B) * (w / B));
              CHECK(np == nb * B * B);
              CHECK(nm > 0 && nm <= np);
            } else {
              CHECK(st == ABCS_EDOMAIN);
              CHECK(strlen(abcs_last_error()) > 0);
            }
          }
  /* malformed descriptors */
  abcs_image bad = img(64, 64, 12, 0.2, ABCS_ZZ);
  CHECK(abcs_image_totals(&bad, NULL, NULL, NULL) == ABCS_EUNSUPPORTED);
  bad = img(64, 64, 16, 0.2, ABCS_ZZ);
  bad.row_pitch = 63;
  CHECK(abcs_image_totals(&bad, NULL, NULL, NULL) == ABCS_EINVAL);
  bad = img(64, 64, 16, NAN, ABCS_DD);
  CHECK(abcs_image_totals(&bad, NULL, NULL, NULL) == ABCS_EDOMAIN);
  CHECK(abcs_image_totals(NULL, NULL, NULL, NULL) == ABCS_EINVAL);

  /* plan creation: bad arguments are refused on the host; a valid batch runs
   * the whole host-side layout (tiles, denoiser and bounds tables) before the
   * device upload, which fails cleanly when there is no device */
  abcs_plan* p = NULL;
  CHECK(abcs_plan_create(NULL, 1, &p) == ABCS_EINVAL && p == NULL);
  CHECK(abcs_plan_create(NULL, 0, NULL) == ABCS_EINVAL);
  CHECK(abcs_plan_create_ex(NULL, 0, 0x80u, &p) == ABCS_EINVAL);
  abcs_image batch[6] = {img(256, 256, 16, 0.25, ABCS_BBV), img(96, 520, 8, 0.3, ABCS_DD),
                         img(128, 120, 32, 0.2, ABCS_ZZ),  img(512, 512, 16, 0.1, ABCS_DD),
                         img(64, 80, 8, 0.5, ABCS_BBV),     img(48, 48, 16, 1.0, ABCS_DD)};
  batch[2].transform = ABCS_WHT;
  for (int i = 1; i < 6; ++i) batch[i].pixel_offset = batch[i - 1].pixel_offset + 512 * 512;
  const int st = abcs_plan_create(batch, 6, &p);
  CHECK(st == ABCS_OK || st == ABCS_EHIP);
  if (st == ABCS_OK) {
    int64_t b = 0, m = 0, px = 0;
    CHECK(abcs_plan_totals(p, &b, &m, &px) == ABCS_OK && b > 0 && m > 0 && px > 0);
    abcs_plan_destroy(p);
  }

  /* launch table */
  abcs_launch_entry e[3] = {{16, ABCS_DCT, ABCS_BF16X3, 1, 2}, {8, ABCS_WHT, ABCS_FP32, 3, 1},
                            {32, ABCS_DCT, ABCS_FP16, 0, 1}};
  CHECK(abcs_set_launch_table(e, 3) == ABCS_OK);
  CHECK(abcs_launch_split(16, ABCS_DCT, ABCS_BF16X3, 1) == 2);
  CHECK(abcs_launch_split(8, ABCS_WHT, ABCS_BF16, 3) == 1);
  abcs_launch_entry badl = {16, ABCS_DCT, ABCS_FP32, 4, 1};
  CHECK(abcs_set_launch_table(&badl, 1) == ABCS_EINVAL);
  CHECK(abcs_launch_split(16, ABCS_DCT, ABCS_BF16X3, 1) == 2);
  CHECK(abcs_set_launch_table(NULL, 0) == ABCS_OK);
  CHECK(abcs_launch_split(16, ABCS_DCT, ABCS_BF16X3, 1) == 0);
  CHECK(abcs_launch_split(12, ABCS_DCT, ABCS_FP32, 0) == ABCS_EINVAL);

  /* constant tables, sizes, identity */
  static double D[32 * 32];
  for (int bi = 0; bi < 3; ++bi) {
    const int B = blocks[bi];
    CHECK(abcs_dct_basis(B, D) == ABCS_OK);
    double s = 0.0;
    for (int j = 0; j < B; ++j) s += D[j] * D[j];
    CHECK(fabs(s - 1.0) < 1e-12);
  }
  CHECK(abcs_dct_basis(12, D) != ABCS_OK);
  CHECK(abcs_cnn_param_count() == 223361);
  CHECK(strlen(abcs_build_id()) > 0);
  printf("%s: %d failed checks\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
