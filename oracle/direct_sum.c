/*
 * Oracle: direct lattice summation of the LGF convolution.  TEST INFRASTRUCTURE ONLY.
 *
 * Computes, for each requested target index n (which may lie outside the source box),
 *     y(n) = dx2 * sum_{m in box} g(n - m) s(m)
 * i.e. the free-space solution L^{-1} s of the discrete Poisson problem written as the discrete
 * convolution of the source with the lattice Green's function (Sec. 2.2, Eq. dpoisson_conv;
 * dx2 = dx^2 carries the dimensional Laplacian of Appendix A).
 *
 * Plain O(N_src * N_tgt) loop, sources visited in fixed z, y, x order, Neumaier-compensated
 * FP64 accumulation.  g is read from a cube gcube[a][b][c] = g(a, b, c) of side gn indexed by the
 * absolute offsets (g is even in each coordinate and symmetric under axis permutations).
 * OpenMP only splits the target list; each target's sum is sequential and deterministic.
 */
#include <math.h>
#include <stdlib.h>
#include <stdint.h>

static inline void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *comp += (*sum - t) + v;
    else
        *comp += (v - t) + *sum;
    *sum = t;
}

/* returns 0 on success, -1 if an offset falls outside the table */
int oracle_lgf_direct(const double *gcube, int64_t gn,
                      const double *src, int64_t nz, int64_t ny, int64_t nx,
                      const int64_t *tgt, int64_t ntgt,
                      double dx2, double *out)
{
    /* gather the nonzero sources once (plain list, box order) */
    int64_t nsrc = 0, total = nz * ny * nx;
    for (int64_t p = 0; p < total; ++p)
        if (src[p] != 0.0) ++nsrc;
    int64_t *sk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nsrc > 0 ? nsrc : 1) * 3);
    double *sv = (double *)malloc(sizeof(double) * (size_t)(nsrc > 0 ? nsrc : 1));
    if (!sk || !sv) { free(sk); free(sv); return -2; }
    int64_t q = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double v = src[(k * ny + j) * nx + i];
                if (v != 0.0) { sk[3 * q] = k; sk[3 * q + 1] = j; sk[3 * q + 2] = i; sv[q] = v; ++q; }
            }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(|: bad)
    for (int64_t t = 0; t < ntgt; ++t) {
        int64_t tk = tgt[3 * t], tj = tgt[3 * t + 1], ti = tgt[3 * t + 2];
        double sum = 0.0, comp = 0.0;
        for (int64_t p = 0; p < nsrc; ++p) {
            int64_t a = llabs(tk - sk[3 * p]), b = llabs(tj - sk[3 * p + 1]), c = llabs(ti - sk[3 * p + 2]);
            if (a >= gn || b >= gn || c >= gn) { bad = 1; continue; }
            neumaier_add(&sum, &comp, gcube[(a * gn + b) * gn + c] * sv[p]);
        }
        out[t] = dx2 * (sum + comp);
    }
    free(sk);
    free(sv);
    return bad ? -1 : 0;
}
