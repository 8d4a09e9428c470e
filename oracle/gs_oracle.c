/*
 * Gray-Scott FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against. Only tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header or constant with the HIP library.
 *
 * What it computes (paper, Section 3.1):
 *   Eq. 1a/1b  dU/dt = Du lap(U) - U V^2 + F (1 - U) + n r
 *              dV/dt = Dv lap(V) + U V^2 - (F + k) V
 *   Eq. 2a/2b  forward Euler in time, Jacobi: level t+1 is computed from
 *              level t only and written to separate arrays.
 *   Eq. 3      7-point Laplacian in normalised units (h = 1), written as in
 *              the paper's Julia kernel (Section 4, kernel listing):
 *              (sum of the six face neighbours - 6 c) / 6, true division.
 *
 * Readings where the paper is silent or ambiguous:
 *   - periodic boundaries in x, y and z, every cell updated;
 *   - x is the fastest index: idx = x + nx (y + ny z);
 *   - the six neighbours are summed pairwise: ((x- + x+) + (y- + y+)) + (z- + z+);
 *   - operations are evaluated left to right as written below, no FMA
 *     contraction (built with -ffp-contract=off);
 *   - the noise term n r is added inside the bracket multiplied by dt (Eq. 2a),
 *     r in (-1, 1) from Philox4x32-10 keyed by (seed, step, cell), see
 *     gso_noise_r; it is skipped entirely when n == 0;
 *   - initial state: u = 1, v = 0 except an axis-aligned cube of side s with
 *     lower corner floor((L - s) / 2) per axis, set to (cube_u, cube_v).
 *
 * Pins: tests/test_oracle_*.py check this file against closed forms (Fourier
 * modes), invariants (mass conservation, fixed point, symmetries), a dense
 * matrix brute force, an independent Python Philox and rocRAND's Philox.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11. Four 32-bit counter words, two 32-bit key words,
 * ten rounds. Each round multiplies words 0 and 2 by the two round
 * multipliers (full 64-bit product), and forms the new words as
 *   new0 = hi(M1*c2) ^ c1 ^ k0,  new1 = lo(M1*c2),
 *   new2 = hi(M0*c0) ^ c3 ^ k1,  new3 = lo(M0*c0);
 * between rounds the key is bumped by the two Weyl constants.           */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void gso_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform noise r(seed, t, idx) in the open interval (-1, 1).
 * Key = (low, high) 32-bit halves of the seed. Counter = (low, high) halves
 * of q = idx / 4, then (low, high) halves of the step index t. The output
 * word idx % 4 is read as a signed 32-bit integer w and mapped to
 * (w + 0.5) * 2^-31, which is exact in FP64.                            */
double gso_noise_r(uint64_t seed, uint64_t t, uint64_t idx)
{
    uint64_t q = idx >> 2;
    uint32_t ctr[4] = { (uint32_t)q, (uint32_t)(q >> 32), (uint32_t)t, (uint32_t)(t >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    gso_philox4x32_10(ctr, key, out);
    int32_t w = (int32_t)out[idx & 3u];
    return ((double)w + 0.5) * (1.0 / 2147483648.0);
}

void gso_noise_field(uint64_t seed, uint64_t t, int64_t n, double *r)
{
    for (int64_t i = 0; i < n; ++i) r[i] = gso_noise_r(seed, t, (uint64_t)i);
}

/* ------------------------------------------------------------------ */
void gso_init_cube(int nx, int ny, int nz, int side, double cu, double cv,
                   double *u, double *v)
{
    int x0 = (nx - side) / 2, y0 = (ny - side) / 2, z0 = (nz - side) / 2;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z);
                int inside = x >= x0 && x < x0 + side && y >= y0 && y < y0 + side &&
                             z >= z0 && z < z0 + side;
                u[c] = inside ? cu : 1.0;
                v[c] = inside ? cv : 0.0;
            }
}

/* Sum of the six face neighbours of cell (x, y, z) with periodic wrap, in the
 * pairwise order ((x- + x+) + (y- + y+)) + (z- + z+).                     */
static double neighbour_sum(const double *f, int nx, int ny, int nz, int x, int y, int z)
{
    int xm = (x + nx - 1) % nx, xp = (x + 1) % nx;
    int ym = (y + ny - 1) % ny, yp = (y + 1) % ny;
    int zm = (z + nz - 1) % nz, zp = (z + 1) % nz;
#define AT(X, Y, Z) f[(size_t)(X) + (size_t)nx * ((size_t)(Y) + (size_t)ny * (size_t)(Z))]
    double sx = AT(xm, y, z) + AT(xp, y, z);
    double sy = AT(x, ym, z) + AT(x, yp, z);
    double sz = AT(x, y, zm) + AT(x, y, zp);
#undef AT
    return (sx + sy) + sz;
}

/* Eq. 3: (sum of six neighbours - 6 c) / 6. */
static double laplacian(const double *f, int nx, int ny, int nz, int x, int y, int z)
{
    double c = f[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z)];
    double s = neighbour_sum(f, nx, ny, nz, x, y, z);
    return (s - 6.0 * c) / 6.0;
}

void gso_laplacian(int nx, int ny, int nz, const double *f, double *out)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                out[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z)] =
                    laplacian(f, nx, ny, nz, x, y, z);
}

/* One Jacobi step t -> t+1 (Eq. 2a/2b with Eq. 1a/1b's source terms).
 * Reads u, v (level t); writes un, vn (level t+1). The noise for this step is
 * keyed by the 0-based index t of the step being taken.                   */
void gso_step(int nx, int ny, int nz, double Du, double Dv, double F, double k,
              double dt, double noise, uint64_t seed, uint64_t t,
              const double *u, const double *v, double *un, double *vn)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z);
                double uc = u[c], vc = v[c];
                double lapu = laplacian(u, nx, ny, nz, x, y, z);
                double lapv = laplacian(v, nx, ny, nz, x, y, z);
                double uvv = uc * (vc * vc);
                double du = (Du * lapu - uvv) + F * (1.0 - uc);
                if (noise != 0.0)
                    du = du + noise * gso_noise_r(seed, t, (uint64_t)c);
                double dv = (Dv * lapv + uvv) - (F + k) * vc;
                un[c] = uc + du * dt;
                vn[c] = vc + dv * dt;
            }
}

/* n_steps steps starting at global step index step0; the result is left in
 * u, v. Returns 0, or -1 if scratch memory could not be allocated.        */
int gso_run(int nx, int ny, int nz, double Du, double Dv, double F, double k,
            double dt, double noise, uint64_t seed, uint64_t step0, int64_t n_steps,
            double *u, double *v)
{
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    double *cu = u, *cv = v, *nu = a, *nv = b;
    for (int64_t s = 0; s < n_steps; ++s) {
        gso_step(nx, ny, nz, Du, Dv, F, k, dt, noise, seed, step0 + (uint64_t)s,
                 cu, cv, nu, nv);
        double *tu = cu, *tv = cv;
        cu = nu; cv = nv; nu = tu; nv = tv;
    }
    if (cu != u) {
        memcpy(u, cu, n * sizeof(double));
        memcpy(v, cv, n * sizeof(double));
    }
    free(a); free(b);
    return 0;
}

/* The same steps evaluated on a w*w*w window of a larger periodic grid
 * (nx, ny, nz), for checking sampled cells of large runs one by one. Window
 * cell (i, j, l) is global cell ((x0 + i) mod nx, (y0 + j) mod ny,
 * (z0 + l) mod nz), and the noise is keyed by the global index. Step s
 * (s = 0, 1, ...) recomputes only cells at least s + 1 cells from the
 * window's faces, whose six neighbours are all still exact; after n_steps
 * the cells at least n_steps from every face hold the exact values.
 * u, v: w^3 doubles each, x fastest, updated in place. Returns 0, or -1 if
 * scratch memory could not be allocated.                                  */
int gso_run_window(int nx, int ny, int nz, int x0, int y0, int z0, int w,
                   double Du, double Dv, double F, double k, double dt, double noise,
                   uint64_t seed, uint64_t step0, int64_t n_steps, double *u, double *v)
{
    size_t n = (size_t)w * (size_t)w * (size_t)w;
    double *nu = (double *)malloc(n * sizeof(double));
    double *nv = (double *)malloc(n * sizeof(double));
    if (!nu || !nv) { free(nu); free(nv); return -1; }
#define W(A, I, J, L) A[(size_t)(I) + (size_t)w * ((size_t)(J) + (size_t)w * (size_t)(L))]
    for (int64_t s = 0; s < n_steps; ++s) {
        int lo = (int)s + 1, hi = w - (int)s - 1;
        memcpy(nu, u, n * sizeof(double));
        memcpy(nv, v, n * sizeof(double));
        for (int l = lo; l < hi; ++l)
            for (int j = lo; j < hi; ++j)
                for (int i = lo; i < hi; ++i) {
                    double uc = W(u, i, j, l), vc = W(v, i, j, l);
                    double su = ((W(u, i - 1, j, l) + W(u, i + 1, j, l)) + (W(u, i, j - 1, l) + W(u, i, j + 1, l)))
                                + (W(u, i, j, l - 1) + W(u, i, j, l + 1));
                    double sv = ((W(v, i - 1, j, l) + W(v, i + 1, j, l)) + (W(v, i, j - 1, l) + W(v, i, j + 1, l)))
                                + (W(v, i, j, l - 1) + W(v, i, j, l + 1));
                    double lapu = (su - 6.0 * uc) / 6.0;
                    double lapv = (sv - 6.0 * vc) / 6.0;
                    double uvv = uc * (vc * vc);
                    double du = (Du * lapu - uvv) + F * (1.0 - uc);
                    if (noise != 0.0) {
                        int gx = ((x0 + i) % nx + nx) % nx;
                        int gy = ((y0 + j) % ny + ny) % ny;
                        int gz = ((z0 + l) % nz + nz) % nz;
                        uint64_t idx = (uint64_t)gx + (uint64_t)nx * ((uint64_t)gy + (uint64_t)ny * (uint64_t)gz);
                        du = du + noise * gso_noise_r(seed, step0 + (uint64_t)s, idx);
                    }
                    double dv = (Dv * lapv + uvv) - (F + k) * vc;
                    W(nu, i, j, l) = uc + du * dt;
                    W(nv, i, j, l) = vc + dv * dt;
                }
        memcpy(u, nu, n * sizeof(double));
        memcpy(v, nv, n * sizeof(double));
    }
#undef W
    free(nu); free(nv);
    return 0;
}

void gso_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int gso_max_threads(void) { return omp_get_max_threads(); }
