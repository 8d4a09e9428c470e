/* Exercises the oracle's entry points on small grids so that the build with
 * -fsanitize=address,undefined can check its memory accesses and arithmetic. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void gso_init_cube(int nx, int ny, int nz, int side, double cu, double cv, double *u, double *v);
int gso_run(int nx, int ny, int nz, double Du, double Dv, double F, double k, double dt, double noise,
            uint64_t seed, uint64_t step0, int64_t n_steps, double *u, double *v);
int gso_run_window(int nx, int ny, int nz, int x0, int y0, int z0, int w, double Du, double Dv, double F, double k,
                   double dt, double noise, uint64_t seed, uint64_t step0, int64_t n_steps, double *u, double *v);
void gso_laplacian(int nx, int ny, int nz, const double *f, double *out);
void gso_noise_field(uint64_t seed, uint64_t t, int64_t n, double *r);

int main(void)
{
    const int dims[3][3] = {{4, 4, 8}, {9, 13, 24}, {16, 16, 16}};
    for (int c = 0; c < 3; ++c) {
        int nz = dims[c][0], ny = dims[c][1], nx = dims[c][2];
        size_t n = (size_t)nx * ny * nz;
        double *u = malloc(n * sizeof(double)), *v = malloc(n * sizeof(double)), *o = malloc(n * sizeof(double));
        gso_init_cube(nx, ny, nz, 3, 0.25, 0.33, u, v);
        if (gso_run(nx, ny, nz, 0.2, 0.1, 0.02, 0.048, 1.0, 0.01, 7, 3, 5, u, v)) return 1;
        gso_laplacian(nx, ny, nz, u, o);
        gso_noise_field(7, 9, (int64_t)n, o);
        free(u); free(v); free(o);
    }
    int w = 10;
    double *uw = malloc((size_t)w * w * w * sizeof(double)), *vw = malloc((size_t)w * w * w * sizeof(double));
    for (int i = 0; i < w * w * w; ++i) { uw[i] = 0.5; vw[i] = 0.25; }
    if (gso_run_window(24, 13, 9, 20, -3, 5, w, 0.2, 0.1, 0.02, 0.048, 1.0, 0.01, 7, 3, 4, uw, vw)) return 1;
    free(uw); free(vw);
    printf("ok\n");
    return 0;
}
