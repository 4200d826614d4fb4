/* Direct rectangle-rule quadrature of the coset convolution on Omega_L.
 *
 * Test infrastructure for the oracle only (never part of the product library).
 *
 * Paper Sec. 5.1, eqs. (oslash) and (f*g): for psi periodized and rho on SE(2),
 *   (psi (/) rho)(x, theta) = (1/2pi) int_Omega f(y, a) sum_l rho(R_{-a}(x - y - l), theta - a) dy da.
 * On the grid x_i = -1/2 + i/Nx (and likewise y, theta_l = 2 pi l / M) the rectangle
 * rule gives weight 1/(Nx Ny M).  The caller tabulates the image-summed kernel
 *   K[l][dc][dj][di] = sum_l rho(R_{-theta_l}((di)/Nx - l1, (dj)/Ny - l2), 2 pi dc / M)
 * for di in [-(Nx-1), Nx-1], dj in [-(Ny-1), Ny-1], dc in [0, M); this routine
 * only performs the O(n^2) sum
 *   out[c][b][a] = 1/(Nx Ny M) sum_{l,j,i} F[l][j][i] K[l][(c-l) mod M][b-j][a-i].
 */
#include <stddef.h>

void quad_sum(const double* F, int nx, int ny, int m, const double* K, double* out)
{
    const int wx = 2 * nx - 1, wy = 2 * ny - 1;
    const double scale = 1.0 / ((double)nx * (double)ny * (double)m);
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < m; ++c) {
        for (int b = 0; b < ny; ++b) {
            for (int a = 0; a < nx; ++a) {
                double acc = 0.0;
                for (int l = 0; l < m; ++l) {
                    int dc = ((c - l) % m + m) % m;
                    const double* Kl = K + ((size_t)l * m + dc) * (size_t)wy * wx;
                    const double* Fl = F + (size_t)l * ny * nx;
                    for (int j = 0; j < ny; ++j) {
                        const double* Kr = Kl + (size_t)(b - j + ny - 1) * wx + (nx - 1) + a;
                        const double* Fr = Fl + (size_t)j * nx;
                        for (int i = 0; i < nx; ++i)
                            acc += Fr[i] * Kr[-i];
                    }
                }
                out[((size_t)c * ny + b) * nx + a] = acc * scale;
            }
        }
    }
}
