/*
 * FP64 CPU oracle for the 3D Yee FDTD leapfrog on a PEC box cavity.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, obviously correct
 * definition that the GPU path is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. It shares
 * no code, header, table or helper with the HIP library.
 *
 * What it computes (paper, Sec. 2 Eq. 2, and Sec. 2.1 with the full
 * algorithm listing and the naive / slicing curl_Hx listings):
 *   each time step = update H from the curl of E (all H nodes), then update E
 *   from the curl of the new H (interior E nodes); tangential E on the six
 *   walls is never written and stays 0 (PEC, Fig. 1b caption, Sec. 4).
 * Readings where the paper is loose:
 *   - Faraday's law carries the minus sign of Eq. 2 (Eq. 1 prints it
 *     without); the H update is H += Ch * (dEy/dz - dEz/dy) for Hx, etc.
 *   - H is advanced first, so with E = E^n, H = H^{n-1/2} on entry a step
 *     leaves E^{n+1}, H^{n+1/2}.
 *   - Differences are one-cell staggered differences with the 1/dx of a cubic
 *     cell folded into the coefficient: Ch = dt/(mu dx), Ce = dt/(eps dx).
 *   - eps and mu are per cell; an edge (E node) takes the mean of the four
 *     cells sharing it, summed as ((a+b)+(c+d))*0.25; a face (H node) the mean
 *     of its two cells. Wall-tangential E nodes and wall-normal H nodes get
 *     coefficient 0 (they never change).
 *
 * Layout: each component is a dense x-fastest array with the staggered extents
 *   Ex (nx, ny+1, nz+1)  Ey (nx+1, ny, nz+1)  Ez (nx+1, ny+1, nz)
 *   Hx (nx+1, ny, nz)    Hy (nx, ny+1, nz)    Hz (nx, ny, nz+1)
 * given as (X, Y, Z); element (i, j, k) sits at i + X*(j + Y*k).
 *
 * Loops over k may run on several OpenMP threads: inside one sweep every node
 * is written once and reads only the other field, so the result does not
 * depend on the thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(a, X, Y, i, j, k) (a)[(size_t)(i) + (size_t)(X) * ((size_t)(j) + (size_t)(Y) * (size_t)(k))]

static int g_threads = 1;

void yee_set_threads(int n) { g_threads = n > 0 ? n : 1; }

int yee_get_threads(void) { return g_threads; }

int yee_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_num_procs();
#else
    return 1;
#endif
}

/* Per-cell material value, 1.0 where the array is absent. */
static double cell(const double *m, int nx, int ny, int i, int j, int k)
{
    return m ? AT(m, nx, ny, i, j, k) : 1.0;
}

/*
 * Ce at every E node: Eq. 2 coefficient dt/eps, read with a per-cell eps.
 * Ex(i,j,k) is the x-edge shared by cells (i, j-1..j, k-1..k).
 */
void yee_coef_e(int nx, int ny, int nz, double dx, double dt, const double *eps,
                double *cex, double *cey, double *cez)
{
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = 0.0;
                if (j > 0 && j < ny && k > 0 && k < nz) {
                    double m = ((cell(eps, nx, ny, i, j - 1, k - 1) + cell(eps, nx, ny, i, j, k - 1)) +
                                (cell(eps, nx, ny, i, j - 1, k) + cell(eps, nx, ny, i, j, k))) * 0.25;
                    c = dt / (dx * m);
                }
                AT(cex, nx, ny + 1, i, j, k) = c;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double c = 0.0;
                if (i > 0 && i < nx && k > 0 && k < nz) {
                    /* y-edge shared by cells (i-1..i, j, k-1..k); cyclic analogue of x */
                    double m = ((cell(eps, nx, ny, i - 1, j, k - 1) + cell(eps, nx, ny, i - 1, j, k)) +
                                (cell(eps, nx, ny, i, j, k - 1) + cell(eps, nx, ny, i, j, k))) * 0.25;
                    c = dt / (dx * m);
                }
                AT(cey, nx + 1, ny, i, j, k) = c;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double c = 0.0;
                if (i > 0 && i < nx && j > 0 && j < ny) {
                    /* z-edge shared by cells (i-1..i, j-1..j, k) */
                    double m = ((cell(eps, nx, ny, i - 1, j - 1, k) + cell(eps, nx, ny, i, j - 1, k)) +
                                (cell(eps, nx, ny, i - 1, j, k) + cell(eps, nx, ny, i, j, k))) * 0.25;
                    c = dt / (dx * m);
                }
                AT(cez, nx + 1, ny + 1, i, j, k) = c;
            }
}

/* Ch at every H node: Hx(i,j,k) is the x-face between cells (i-1,j,k) and (i,j,k). */
void yee_coef_h(int nx, int ny, int nz, double dx, double dt, const double *mu,
                double *chx, double *chy, double *chz)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double c = 0.0;
                if (i > 0 && i < nx) {
                    double m = (cell(mu, nx, ny, i - 1, j, k) + cell(mu, nx, ny, i, j, k)) * 0.5;
                    c = dt / (dx * m);
                }
                AT(chx, nx + 1, ny, i, j, k) = c;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = 0.0;
                if (j > 0 && j < ny) {
                    double m = (cell(mu, nx, ny, i, j - 1, k) + cell(mu, nx, ny, i, j, k)) * 0.5;
                    c = dt / (dx * m);
                }
                AT(chy, nx, ny + 1, i, j, k) = c;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = 0.0;
                if (k > 0 && k < nz) {
                    double m = (cell(mu, nx, ny, i, j, k - 1) + cell(mu, nx, ny, i, j, k)) * 0.5;
                    c = dt / (dx * m);
                }
                AT(chz, nx, ny, i, j, k) = c;
            }
}

/*
 * Faraday half of the leapfrog (Eq. 2, right column), every H node.
 * Hx follows the naive curl_Hx listing with Dy = Dz = dx folded into Ch.
 */
void yee_update_h(int nx, int ny, int nz,
                  double *hx, double *hy, double *hz,
                  const double *ex, const double *ey, const double *ez,
                  const double *chx, const double *chy, const double *chz)
{
    const int ExX = nx, ExY = ny + 1;
    const int EyX = nx + 1, EyY = ny;
    const int EzX = nx + 1, EzY = ny + 1;
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i)
                AT(hx, nx + 1, ny, i, j, k) += AT(chx, nx + 1, ny, i, j, k) *
                    ((AT(ey, EyX, EyY, i, j, k + 1) - AT(ey, EyX, EyY, i, j, k)) -
                     (AT(ez, EzX, EzY, i, j + 1, k) - AT(ez, EzX, EzY, i, j, k)));
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(hy, nx, ny + 1, i, j, k) += AT(chy, nx, ny + 1, i, j, k) *
                    ((AT(ez, EzX, EzY, i + 1, j, k) - AT(ez, EzX, EzY, i, j, k)) -
                     (AT(ex, ExX, ExY, i, j, k + 1) - AT(ex, ExX, ExY, i, j, k)));
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(hz, nx, ny, i, j, k) += AT(chz, nx, ny, i, j, k) *
                    ((AT(ex, ExX, ExY, i, j + 1, k) - AT(ex, ExX, ExY, i, j, k)) -
                     (AT(ey, EyX, EyY, i + 1, j, k) - AT(ey, EyX, EyY, i, j, k)));
}

/* Ampere half (Eq. 2, left column, J = 0), interior E nodes only (PEC walls untouched). */
void yee_update_e(int nx, int ny, int nz,
                  double *ex, double *ey, double *ez,
                  const double *hx, const double *hy, const double *hz,
                  const double *cex, const double *cey, const double *cez)
{
    const int HxX = nx + 1, HxY = ny;
    const int HyX = nx, HyY = ny + 1;
    const int HzX = nx, HzY = ny;
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 1; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(ex, nx, ny + 1, i, j, k) += AT(cex, nx, ny + 1, i, j, k) *
                    ((AT(hz, HzX, HzY, i, j, k) - AT(hz, HzX, HzY, i, j - 1, k)) -
                     (AT(hy, HyX, HyY, i, j, k) - AT(hy, HyX, HyY, i, j, k - 1)));
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                AT(ey, nx + 1, ny, i, j, k) += AT(cey, nx + 1, ny, i, j, k) *
                    ((AT(hx, HxX, HxY, i, j, k) - AT(hx, HxX, HxY, i, j, k - 1)) -
                     (AT(hz, HzX, HzY, i, j, k) - AT(hz, HzX, HzY, i - 1, j, k)));
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                AT(ez, nx + 1, ny + 1, i, j, k) += AT(cez, nx + 1, ny + 1, i, j, k) *
                    ((AT(hy, HyX, HyY, i, j, k) - AT(hy, HyX, HyY, i - 1, j, k)) -
                     (AT(hx, HxX, HxY, i, j, k) - AT(hx, HxX, HxY, i, j - 1, k)));
}

/* Zero tangential E on the six walls (PEC). */
void yee_pec(int nx, int ny, int nz, double *ex, double *ey, double *ez)
{
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                if (j == 0 || j == ny || k == 0 || k == nz)
                    AT(ex, nx, ny + 1, i, j, k) = 0.0;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i)
                if (i == 0 || i == nx || k == 0 || k == nz)
                    AT(ey, nx + 1, ny, i, j, k) = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i)
                if (i == 0 || i == nx || j == 0 || j == ny)
                    AT(ez, nx + 1, ny + 1, i, j, k) = 0.0;
}

/* The full algorithm: n times (update H, H boundary (nothing to do), update E, E boundary). */
void yee_run(int nx, int ny, int nz,
             double *ex, double *ey, double *ez, double *hx, double *hy, double *hz,
             const double *cex, const double *cey, const double *cez,
             const double *chx, const double *chy, const double *chz, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) {
        yee_update_h(nx, ny, nz, hx, hy, hz, ex, ey, ez, chx, chy, chz);
        yee_update_e(nx, ny, nz, ex, ey, ez, hx, hy, hz, cex, cey, cez);
    }
}

/*
 * Rectangular cells dx x dy x dz: Eq. 2 with each difference divided by its
 * own spacing, as the naive curl_Hx listing writes with Dy and Dz, in
 * physical field values. Coefficients are ch = dt/mu and ce = dt/eps with no
 * spacing folded in (yee_coef_h / yee_coef_e with dx = 1 produce them).
 */
void yee_update_h_rect(int nx, int ny, int nz,
                       double *hx, double *hy, double *hz,
                       const double *ex, const double *ey, const double *ez,
                       const double *chx, const double *chy, const double *chz,
                       double dx, double dy, double dz)
{
    const int ExX = nx, ExY = ny + 1;
    const int EyX = nx + 1, EyY = ny;
    const int EzX = nx + 1, EzY = ny + 1;
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i)
                AT(hx, nx + 1, ny, i, j, k) += AT(chx, nx + 1, ny, i, j, k) *
                    ((AT(ey, EyX, EyY, i, j, k + 1) - AT(ey, EyX, EyY, i, j, k)) / dz -
                     (AT(ez, EzX, EzY, i, j + 1, k) - AT(ez, EzX, EzY, i, j, k)) / dy);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(hy, nx, ny + 1, i, j, k) += AT(chy, nx, ny + 1, i, j, k) *
                    ((AT(ez, EzX, EzY, i + 1, j, k) - AT(ez, EzX, EzY, i, j, k)) / dx -
                     (AT(ex, ExX, ExY, i, j, k + 1) - AT(ex, ExX, ExY, i, j, k)) / dz);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(hz, nx, ny, i, j, k) += AT(chz, nx, ny, i, j, k) *
                    ((AT(ex, ExX, ExY, i, j + 1, k) - AT(ex, ExX, ExY, i, j, k)) / dy -
                     (AT(ey, EyX, EyY, i + 1, j, k) - AT(ey, EyX, EyY, i, j, k)) / dx);
}

void yee_update_e_rect(int nx, int ny, int nz,
                       double *ex, double *ey, double *ez,
                       const double *hx, const double *hy, const double *hz,
                       const double *cex, const double *cey, const double *cez,
                       double dx, double dy, double dz)
{
    const int HxX = nx + 1, HxY = ny;
    const int HyX = nx, HyY = ny + 1;
    const int HzX = nx, HzY = ny;
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 1; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(ex, nx, ny + 1, i, j, k) += AT(cex, nx, ny + 1, i, j, k) *
                    ((AT(hz, HzX, HzY, i, j, k) - AT(hz, HzX, HzY, i, j - 1, k)) / dy -
                     (AT(hy, HyX, HyY, i, j, k) - AT(hy, HyX, HyY, i, j, k - 1)) / dz);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                AT(ey, nx + 1, ny, i, j, k) += AT(cey, nx + 1, ny, i, j, k) *
                    ((AT(hx, HxX, HxY, i, j, k) - AT(hx, HxX, HxY, i, j, k - 1)) / dz -
                     (AT(hz, HzX, HzY, i, j, k) - AT(hz, HzX, HzY, i - 1, j, k)) / dx);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                AT(ez, nx + 1, ny + 1, i, j, k) += AT(cez, nx + 1, ny + 1, i, j, k) *
                    ((AT(hy, HyX, HyY, i, j, k) - AT(hy, HyX, HyY, i - 1, j, k)) / dx -
                     (AT(hx, HxX, HxY, i, j, k) - AT(hx, HxX, HxY, i, j - 1, k)) / dy);
}

void yee_run_rect(int nx, int ny, int nz,
                  double *ex, double *ey, double *ez, double *hx, double *hy, double *hz,
                  const double *cex, const double *cey, const double *cez,
                  const double *chx, const double *chy, const double *chz,
                  double dx, double dy, double dz, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) {
        yee_update_h_rect(nx, ny, nz, hx, hy, hz, ex, ey, ez, chx, chy, chz, dx, dy, dz);
        yee_update_e_rect(nx, ny, nz, ex, ey, ez, hx, hy, hz, cex, cey, cez, dx, dy, dz);
    }
}

/*
 * Discrete energy W^n = sum E^2/Ce + sum H^{n-1/2} . H^{n+1/2} / Ch over nodes
 * with a nonzero coefficient. The leapfrog conserves it exactly in exact
 * arithmetic because the E curl is minus the transpose of the H curl.
 * H^{n+1/2} is formed here node by node from the state (E^n, H^{n-1/2}).
 * Also returns sum E^2 and sum H^2 in out[1], out[2].
 */
void yee_energy(int nx, int ny, int nz,
                const double *ex, const double *ey, const double *ez,
                const double *hx, const double *hy, const double *hz,
                const double *cex, const double *cey, const double *cez,
                const double *chx, const double *chy, const double *chz, double out[3])
{
    const int ExX = nx, ExY = ny + 1, EyX = nx + 1, EyY = ny, EzX = nx + 1, EzY = ny + 1;
    double we = 0.0, wh = 0.0, se = 0.0, sh = 0.0;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double e = AT(ex, ExX, ExY, i, j, k), c = AT(cex, ExX, ExY, i, j, k);
                se += e * e;
                if (c != 0.0) we += e * e / c;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double e = AT(ey, EyX, EyY, i, j, k), c = AT(cey, EyX, EyY, i, j, k);
                se += e * e;
                if (c != 0.0) we += e * e / c;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double e = AT(ez, EzX, EzY, i, j, k), c = AT(cez, EzX, EzY, i, j, k);
                se += e * e;
                if (c != 0.0) we += e * e / c;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double h = AT(hx, nx + 1, ny, i, j, k), c = AT(chx, nx + 1, ny, i, j, k);
                sh += h * h;
                if (c != 0.0) {
                    double hn = h + c * ((AT(ey, EyX, EyY, i, j, k + 1) - AT(ey, EyX, EyY, i, j, k)) -
                                         (AT(ez, EzX, EzY, i, j + 1, k) - AT(ez, EzX, EzY, i, j, k)));
                    wh += h * hn / c;
                }
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double h = AT(hy, nx, ny + 1, i, j, k), c = AT(chy, nx, ny + 1, i, j, k);
                sh += h * h;
                if (c != 0.0) {
                    double hn = h + c * ((AT(ez, EzX, EzY, i + 1, j, k) - AT(ez, EzX, EzY, i, j, k)) -
                                         (AT(ex, ExX, ExY, i, j, k + 1) - AT(ex, ExX, ExY, i, j, k)));
                    wh += h * hn / c;
                }
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double h = AT(hz, nx, ny, i, j, k), c = AT(chz, nx, ny, i, j, k);
                sh += h * h;
                if (c != 0.0) {
                    double hn = h + c * ((AT(ex, ExX, ExY, i, j + 1, k) - AT(ex, ExX, ExY, i, j, k)) -
                                         (AT(ey, EyX, EyY, i + 1, j, k) - AT(ey, EyX, EyY, i, j, k)));
                    wh += h * hn / c;
                }
            }
    out[0] = we + wh;
    out[1] = se;
    out[2] = sh;
}

/*
 * Discrete divergence per cell of H (ch == NULL) or of B = H/Ch (ch given; nodes
 * with Ch = 0 count as 0, they never change):
 * (Fx[i+1]-Fx[i]) + (Fy[j+1]-Fy[j]) + (Fz[k+1]-Fz[k]); out is nx*ny*nz, x-fastest.
 * The H update adds a discrete curl of E to B, whose divergence is zero.
 */
static double bval(const double *h, const double *c, size_t at)
{
    if (!c)
        return h[at];
    return c[at] != 0.0 ? h[at] / c[at] : 0.0;
}

void yee_div_h(int nx, int ny, int nz, const double *hx, const double *hy, const double *hz,
               const double *chx, const double *chy, const double *chz, double *out)
{
#define IX(X, Y, i, j, k) ((size_t)(i) + (size_t)(X) * ((size_t)(j) + (size_t)(Y) * (size_t)(k)))
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                AT(out, nx, ny, i, j, k) =
                    (bval(hx, chx, IX(nx + 1, ny, i + 1, j, k)) - bval(hx, chx, IX(nx + 1, ny, i, j, k))) +
                    (bval(hy, chy, IX(nx, ny + 1, i, j + 1, k)) - bval(hy, chy, IX(nx, ny + 1, i, j, k))) +
                    (bval(hz, chz, IX(nx, ny, i, j, k + 1)) - bval(hz, chz, IX(nx, ny, i, j, k)));
#undef IX
}

/*
 * Discrete divergence of D = E/Ce at every interior node (i,j,k), 1 <= i < nx
 * etc.; out is (nx-1)*(ny-1)*(nz-1), x-fastest. The E update adds a discrete
 * curl to D, whose divergence is zero, so this stays constant in time.
 */
void yee_div_d(int nx, int ny, int nz, const double *ex, const double *ey, const double *ez,
               const double *cex, const double *cey, const double *cez, double *out)
{
    const int ExX = nx, ExY = ny + 1, EyX = nx + 1, EyY = ny, EzX = nx + 1, EzY = ny + 1;
#define D(a, c, X, Y, i, j, k) (AT(c, X, Y, i, j, k) != 0.0 ? AT(a, X, Y, i, j, k) / AT(c, X, Y, i, j, k) : 0.0)
    for (int k = 1; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 1; i < nx; ++i)
                AT(out, nx - 1, ny - 1, i - 1, j - 1, k - 1) =
                    (D(ex, cex, ExX, ExY, i, j, k) - D(ex, cex, ExX, ExY, i - 1, j, k)) +
                    (D(ey, cey, EyX, EyY, i, j, k) - D(ey, cey, EyX, EyY, i, j - 1, k)) +
                    (D(ez, cez, EzX, EzY, i, j, k) - D(ez, cez, EzX, EzY, i, j, k - 1));
#undef D
}
