// Active-domain classification on the host (Sec. 4.2, 4.3): from the block weights mu, nu the weight
// function W = max(mu / mu_global, nu / nu_global) (Eq. weight_fun), the support and solution blocks
// {W > eps} (Eqs. d_supp, d_soln) and the expanded solution blocks, every block at most n_xb blocks
// from a solution block along each axis (Eq. def_xsoln), on the box's block grid.
#include <algorithm>

#include "kernels.h"

namespace nslgf {

void classify_blocks_host(const double* mu, const double* nu, int bx, int by, int bz, double eps_supp, double eps_soln,
                          int n_xb, double* W, unsigned char* supp, unsigned char* soln, unsigned char* xsoln) {
    const long long n = (long long)bx * by * bz;
    double mg = 0.0, ng = 0.0;
    for (long long b = 0; b < n; ++b) {
        mg = std::max(mg, mu[b]);
        ng = std::max(ng, nu[b]);
    }
    for (long long b = 0; b < n; ++b) {
        const double w = std::max(mg > 0.0 ? mu[b] / mg : 0.0, ng > 0.0 ? nu[b] / ng : 0.0);
        if (W) W[b] = w;
        supp[b] = w > eps_supp ? 1 : 0;
        soln[b] = w > eps_soln ? 1 : 0;
        xsoln[b] = 0;
    }
    for (int k = 0; k < bz; ++k)
        for (int j = 0; j < by; ++j)
            for (int i = 0; i < bx; ++i) {
                if (!soln[((long long)k * by + j) * bx + i]) continue;
                for (int kk = std::max(0, k - n_xb); kk <= std::min(bz - 1, k + n_xb); ++kk)
                    for (int jj = std::max(0, j - n_xb); jj <= std::min(by - 1, j + n_xb); ++jj)
                        for (int ii = std::max(0, i - n_xb); ii <= std::min(bx - 1, i + n_xb); ++ii)
                            xsoln[((long long)kk * by + jj) * bx + ii] = 1;
            }
}

}  // namespace nslgf
