/* Test driver: runs the CPU oracle's whole method on one pair read from a file, so that the
 * test-suite can build the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Input file: pgmo_params, then int32 w, h, then two w*h*3 RGB images. Output file: n_evals
 * (uint64), n_inliers (int32), the forward and backward matches of both schedules. */
#include <stdio.h>
#include <stdlib.h>

#include "pgm_oracle.h"

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 3;
    pgmo_params p;
    int32_t wh[2];
    if (fread(&p, sizeof p, 1, f) != 1 || fread(wh, 4, 2, f) != 2) return 4;
    size_t bytes = (size_t)wh[0] * wh[1] * 3;
    uint8_t* img1 = malloc(bytes);
    uint8_t* img2 = malloc(bytes);
    if (fread(img1, 1, bytes, f) != bytes || fread(img2, 1, bytes, f) != bytes) return 5;
    fclose(f);
    int32_t lw[PGMO_MAX_LEVELS], lh[PGMO_MAX_LEVELS], lnx[PGMO_MAX_LEVELS], lny[PGMO_MAX_LEVELS];
    if (pgmo_geometry(&p, wh[0], wh[1], lw, lh, lnx, lny) != 0) return 6;
    size_t n = (size_t)lnx[0] * lny[0];
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 7;
    for (int schedule = PGMO_SYNC; schedule <= PGMO_SCAN; schedule++) {
        pgmo_match_t* fwd = malloc(n * sizeof *fwd);
        pgmo_match_t* bwd = malloc(n * sizeof *bwd);
        pgmo_match_t* cmp = malloc(n * sizeof *cmp);
        int32_t n_in = 0;
        uint64_t nev = 0;
        if (pgmo_match(&p, img1, img2, wh[0], wh[1], wh[0] * 3, schedule, fwd, bwd, &n_in, cmp, NULL, &nev) != 0)
            return 8;
        fwrite(&nev, 8, 1, o);
        fwrite(&n_in, 4, 1, o);
        fwrite(fwd, sizeof *fwd, n, o);
        fwrite(bwd, sizeof *bwd, n, o);
        free(fwd); free(bwd); free(cmp);
    }
    fclose(o);
    free(img1); free(img2);
    return 0;
}
