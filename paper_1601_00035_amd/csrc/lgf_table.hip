// LGF table builder (Appendix B) and the padded kernel spectrum used by the FFT convolution.
//
// g(n) = -int_0^inf e^{-6t} I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt is evaluated two ways:
//  * near field (|n| < kNearR): the integrand is separable, so with nodes t_k and weights W_k of a
//    quadrature in s = ln t, g(n) = -(sum_k W_k a_k[n1] a_k[n2] a_k[n3] + tail), where
//    a_k[m] = e^{-2 t_k} I_m(2 t_k) is one vector per node.  The vectors come from the power series
//    (small argument), Miller's normalised backward recurrence with e^{-z}(I_0 + 2 sum I_m)(z) = 1
//    (moderate argument) or the Hankel large-argument series.  Gauss-Legendre panels of width 1/2
//    cover s in [-42, ln 1e11]; the rest of the integral beyond T = 1e11 is the closed-form integral
//    of the two leading Hankel terms.
//  * far field (|n| >= kNearR): the expansion of g in powers of 1/|n| (the two printed terms carried to
//    seven orders; coefficients in lgf_asym_coefs.h).
// Both agree with an independent 1e-17 reference to about 1e-15 relative (double rounding).
#include <cmath>
#include <vector>

#include "kernels.h"
#include "lgf_asym_coefs.h"

namespace nslgf {

constexpr int kNearR = 40;            // |n| < kNearR uses the quadrature
constexpr int kNearN = kNearR;        // components 0..kNearR-1
constexpr double kSMin = -42.0;
constexpr double kSMax = 25.328436022934504;  // ln(1e11)
constexpr double kPanel = 0.5;
constexpr int kGL = 16;

struct Quadrature {
    std::vector<double> t, w;
};

static void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w) {
    x.resize(n);
    w.resize(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L)), pp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1);
            long double dz = p1 / pp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * pp * pp);
    }
}

static const Quadrature& quadrature() {
    static Quadrature q = [] {
        Quadrature r;
        std::vector<long double> x, w;
        gauss_legendre(kGL, x, w);
        const int panels = (int)ceil((kSMax - kSMin) / kPanel - 1e-9);
        const long double h = (kSMax - kSMin) / (long double)panels;
        for (int p = 0; p < panels; ++p) {
            const long double mid = kSMin + (p + 0.5L) * h;
            for (int i = 0; i < kGL; ++i) {
                const long double s = mid + 0.5L * h * x[i];
                const long double t = expl(s);
                r.t.push_back((double)t);
                r.w.push_back((double)(w[i] * 0.5L * h * t));
            }
        }
        return r;
    }();
    return q;
}

// a[m] = e^{-z} I_m(z), m = 0..nmax, z = 2t.
__host__ __device__ static void bessel_scaled_vec(double t, double* a, int nmax) {
    const double z = 2.0 * t;
    const double zh = fmax(1000.0, 30.0 * nmax * nmax);
    if (z < 2.0) {
        // power series: e^{-z} sum_k (z/2)^{2k+m} / (k! (k+m)!)
        const double h = 0.5 * z, h2 = h * h, ez = exp(-z);
        double lead = 1.0;  // (z/2)^m / m!
        for (int m = 0; m <= nmax; ++m) {
            if (m > 0) lead *= h / m;
            double term = lead, sum = lead;
            for (int k = 1; k < 40 && term > 1e-40 * sum; ++k) {
                term *= h2 / ((double)k * (double)(k + m));
                sum += term;
            }
            a[m] = ez * sum;
        }
    } else if (z < zh) {
        const int nstart = nmax + 30 + (int)(12.0 * sqrt(z));
        double fnext = 0.0, f = 1e-30, sum = 0.0;
        for (int n = nstart; n >= 1; --n) {
            const double fprev = fnext + (2.0 * n / z) * f;
            sum += 2.0 * f;
            if (n <= nmax) a[n] = f;
            fnext = f;
            f = fprev;
            if (f > 1e200) {
                f *= 1e-200;
                fnext *= 1e-200;
                sum *= 1e-200;
                for (int m = n; m <= nmax; ++m) a[m] *= 1e-200;
            }
        }
        sum += f;
        a[0] = f;
        const double inv = 1.0 / sum;
        for (int m = 0; m <= nmax; ++m) a[m] *= inv;
    } else {
        // e^{-z} I_m(z) ~ (2 pi z)^{-1/2} sum_k (-1)^k prod_{i<=k} (4m^2 - (2i-1)^2) / (i 8 z)
        const double pre = 1.0 / sqrt(2.0 * 3.14159265358979323846 * z);
        for (int m = 0; m <= nmax; ++m) {
            const double mu = 4.0 * m * m;
            double term = 1.0, sum = 1.0;
            for (int k = 1; k < 30; ++k) {
                const double q = (double)(2 * k - 1);
                term *= -(mu - q * q) / (8.0 * z * k);
                sum += term;
                if (fabs(term) < 1e-22) break;
            }
            a[m] = pre * sum;
        }
    }
}

// Closed-form integral over [T, inf) of the product of the two leading Hankel terms, plus the
// negligible [0, t_min] piece at the origin.
__host__ __device__ static double near_tail(int n1, int n2, int n3, double T, double tmin) {
    const double c = ((4.0 * n1 * n1 - 1) + (4.0 * n2 * n2 - 1) + (4.0 * n3 * n3 - 1)) / 16.0;
    const double k = 1.0 / (4.0 * 3.14159265358979323846 * sqrt(4.0 * 3.14159265358979323846));  // (4 pi)^{-3/2}
    double v = k * (2.0 / sqrt(T) - (2.0 / 3.0) * c / (T * sqrt(T)));
    if (n1 == 0 && n2 == 0 && n3 == 0) v += tmin;
    return v;
}

__host__ __device__ static double lgf_far(int a, int b, int c) {
    const double x = a, y = b, z = c;
    const double r2 = x * x + y * y + z * z, r = sqrt(r2);
    const double u1 = x * x / r2, u2 = y * y / r2, u3 = z * z / r2;
    const double e2 = u1 * u2 + u1 * u3 + u2 * u3, e3 = u1 * u2 * u3;
    double q[kLgfAsymOrders];
    for (int p = 0; p < kLgfAsymOrders; ++p) q[p] = 0.0;
    for (int i = 0; i < kLgfAsymTerms; ++i) {
        double m = kLgfAsym[i].c;
        for (int j = 0; j < kLgfAsym[i].j; ++j) m *= e2;
        for (int l = 0; l < kLgfAsym[i].l; ++l) m *= e3;
        q[kLgfAsym[i].p] += m;
    }
    // sum_p r^{-1-2p} Q_p / pi, highest order first
    const double ir2 = 1.0 / r2;
    double s = 0.0;
    for (int p = kLgfAsymOrders - 1; p >= 0; --p) s = s * ir2 + q[p];
    return s / (r * 3.14159265358979323846);
}

// Neumaier-compensated near-field sum for one entry.
__host__ __device__ static double near_sum(const double* vec, const double* w, int nodes, int stride, int a, int b,
                                           int c) {
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < nodes; ++k) {
        const double* v = vec + (long long)k * stride;
        const double term = w[k] * v[a] * v[b] * v[c];
        const double tt = s + term;
        comp += (fabs(s) >= fabs(term)) ? (s - tt) + term : (term - tt) + s;
        s = tt;
    }
    return s + comp;
}

__global__ void k_bessel_vectors(const double* t, int nodes, double* vec, int stride, int nmax) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nodes) return;
    bessel_scaled_vec(t[k], vec + (long long)k * stride, nmax);
}

// near[a][b][c] for kNearN > a >= b >= c >= 0 (other entries untouched)
__global__ void k_near_table(const double* vec, const double* w, int nodes, int stride, double T, double tmin,
                             double* near) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kNearN * kNearN * kNearN) return;
    const int a = idx / (kNearN * kNearN), b = (idx / kNearN) % kNearN, c = idx % kNearN;
    if (!(a >= b && b >= c)) return;
    if (a * a + b * b + c * c >= kNearR * kNearR) return;
    near[idx] = -(near_sum(vec, w, nodes, stride, a, b, c) + near_tail(a, b, c, T, tmin));
}

__device__ __forceinline__ void sort3(int& a, int& b, int& c) {
    int t;
    if (a < b) { t = a; a = b; b = t; }
    if (b < c) { t = b; b = c; c = t; }
    if (a < b) { t = a; a = b; b = t; }
}

// Even padded kernel K[iz][iy][ix] = g(|ix|_P, |iy|_P, |iz|_P), |i|_P = min(i, P - i).
__global__ void k_scatter_kernel(const double* near, int Px, int Py, int Pz, double* K) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)Px * Py * Pz;
    if (idx >= total) return;
    const int ix = (int)(idx % Px);
    const int iy = (int)((idx / Px) % Py);
    const int iz = (int)(idx / ((long long)Px * Py));
    int a = min(ix, Px - ix), b = min(iy, Py - iy), c = min(iz, Pz - iz);
    sort3(a, b, c);
    double g;
    if (a * a + b * b + c * c < kNearR * kNearR)
        g = near[(a * kNearN + b) * kNearN + c];
    else
        g = lgf_far(a, b, c);
    K[idx] = g;
}

template <typename T>
__global__ void k_extract(const double2* spec, int Px, int Py, int Pz, long long XP, double scale, int tb, int tiles,
                          T* khat) {
    // khat[ky][tile][kz][c], ky <= Py/2, kz <= Pz/2
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nkz = Pz / 2 + 1, nky = Py / 2 + 1;
    const long long total = (long long)nky * tiles * nkz * tb;
    if (idx >= total) return;
    const int c = (int)(idx % tb);
    const int kz = (int)((idx / tb) % nkz);
    const int tile = (int)((idx / ((long long)tb * nkz)) % tiles);
    const int ky = (int)(idx / ((long long)tb * nkz * tiles));
    const int kx = tile * tb + c;
    double v = 0.0;
    if (kx <= Px / 2) v = spec[((long long)kz * Py + ky) * XP + kx].x * scale;
    khat[idx] = (T)v;
}

// ---------------------------------------------------------------------------------------------------
double lgf_value_host(int n1, int n2, int n3) {
    int a = abs(n1), b = abs(n2), c = abs(n3);
    int t;
    if (a < b) { t = a; a = b; b = t; }
    if (b < c) { t = b; b = c; c = t; }
    if (a < b) { t = a; a = b; b = t; }
    if (a * a + b * b + c * c >= kNearR * kNearR) return lgf_far(a, b, c);
    const Quadrature& q = quadrature();
    const int nodes = (int)q.t.size();
    std::vector<double> vec((size_t)nodes * kNearN);
    for (int k = 0; k < nodes; ++k) bessel_scaled_vec(q.t[k], vec.data() + (size_t)k * kNearN, kNearN - 1);
    return -(near_sum(vec.data(), q.w.data(), nodes, kNearN, a, b, c) + near_tail(a, b, c, exp(kSMax), exp(kSMin)));
}

int build_padded_lgf(int Px, int Py, int Pz, double* dev_kernel, hipStream_t s) {
    const Quadrature& q = quadrature();
    const int nodes = (int)q.t.size();
    double *dt = nullptr, *dw = nullptr, *dvec = nullptr, *dnear = nullptr;
    const size_t near_n = (size_t)kNearN * kNearN * kNearN;
    int rc = NSLGF_OK;
    if (hipMalloc(&dt, nodes * sizeof(double)) != hipSuccess || hipMalloc(&dw, nodes * sizeof(double)) != hipSuccess ||
        hipMalloc(&dvec, (size_t)nodes * kNearN * sizeof(double)) != hipSuccess ||
        hipMalloc(&dnear, near_n * sizeof(double)) != hipSuccess) {
        set_error("hipMalloc(lgf table scratch) failed");
        rc = NSLGF_ENOMEM;
    }
    if (rc == NSLGF_OK) {
        hipMemcpyAsync(dt, q.t.data(), nodes * sizeof(double), hipMemcpyHostToDevice, s);
        hipMemcpyAsync(dw, q.w.data(), nodes * sizeof(double), hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_bessel_vectors, dim3(ceil_div(nodes, 64)), dim3(64), 0, s, dt, nodes, dvec, kNearN,
                           kNearN - 1);
        hipLaunchKernelGGL(k_near_table, dim3(ceil_div(near_n, 256)), dim3(256), 0, s, dvec, dw, nodes, kNearN,
                           exp(kSMax), exp(kSMin), dnear);
        const long long total = (long long)Px * Py * Pz;
        hipLaunchKernelGGL(k_scatter_kernel, dim3(ceil_div(total, 256)), dim3(256), 0, s, dnear, Px, Py, Pz,
                           dev_kernel);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            set_error("lgf table kernels failed");
            rc = NSLGF_EHIP;
        }
    }
    hipFree(dt);
    hipFree(dw);
    hipFree(dvec);
    hipFree(dnear);
    return rc;
}

int extract_spectrum(const void* spec, int Px, int Py, int Pz, long long XP, double scale, int tb, int tiles, int dtype,
                     void* khat, hipStream_t s) {
    const long long total = (long long)(Py / 2 + 1) * tiles * (Pz / 2 + 1) * tb;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_extract<float>, dim3(ceil_div(total, 256)), dim3(256), 0, s, (const double2*)spec, Px, Py,
                           Pz, XP, scale, tb, tiles, (float*)khat);
    else
        hipLaunchKernelGGL(k_extract<double>, dim3(ceil_div(total, 256)), dim3(256), 0, s, (const double2*)spec, Px,
                           Py, Pz, XP, scale, tb, tiles, (double*)khat);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

}  // namespace nslgf
