// two_stream.hip -- clear-sky two-stream column that sets the flux entering
// the top of the ray tracer's domain (sec. 2.3, initialisation paragraph).
// C ABI declared in include/rt3d.h (rt3d_two_stream).
//
// One lane per column (a column is typically one g-point's clear-sky
// profile): the work is a few hundred layers per column, so the kernel is a
// short latency-bound chain, run once per radiation call.  FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rt3d.h"

namespace {

constexpr double kKFloor = 1e-12;     // eigenvalue floor (conservative scattering)
constexpr double kResonance = 1e-5;   // |1 - k^2 mu0^2| below this: resonant layer
constexpr double kShift = 1e-5;       // relative mu0 shift around a resonance

struct LayerRT {
    double R, T;        // diffuse reflectance / transmittance (either face)
    double Rdir, Tdir;  // direct beam -> diffuse up at the top / down at the bottom
    double Tb;          // unscattered direct transmittance
};

// Direct-beam terms for the sun at cosine mu: particular solution
// (U, D) = (a, b) exp(-tau/mu) for unit direct horizontal flux at the top,
// plus the source-free solution that removes its diffuse flux entering at
// the top (-b) and at the bottom (-a exp(-tau/mu)), which the layer reflects
// and transmits with R and T.
__device__ void direct_terms(double tau, double w, double g, double g1, double g2, double k, double R, double T,
                             double mu, double* Rdir, double* Tdir) {
    const double g3 = 0.25 * (2.0 - 3.0 * mu * g);
    const double g4 = 1.0 - g3;
    const double d = 1.0 - k * k * mu * mu;
    const double a = w * (g3 * (1.0 - g1 * mu) - g2 * g4 * mu) / d;
    const double b = -w * (g4 * (1.0 + g1 * mu) + g2 * g3 * mu) / d;
    const double tb = exp(-tau / mu);
    *Rdir = a - R * b - T * a * tb;
    *Tdir = b * tb - T * b - R * a * tb;
}

// One homogeneous layer with PIFM coefficients.
__device__ LayerRT layer_rt(double tau, double w, double g, double mu0) {
    const double g1 = 0.25 * (8.0 - w * (5.0 + 3.0 * g));
    const double g2 = 0.75 * w * (1.0 - g);
    const double k = fmax(sqrt(fmax((g1 - g2) * (g1 + g2), 0.0)), kKFloor);
    // source-free solution: modes exp(+-k tau); E = exp(-k tau), X = 1 - E^2
    const double e = exp(-k * tau);
    const double x = -expm1(-2.0 * k * tau);
    const double den = k * (1.0 + e * e) + g1 * x;
    LayerRT L;
    L.R = g2 * x / den;
    L.T = 2.0 * k * e / den;
    if (fabs(1.0 - k * k * mu0 * mu0) < kResonance) {
        // singular particular solution, smooth result: mean of both sides
        // (error O(kShift^2) from the mean; just outside the window the
        // closed form loses about eps / kResonance to cancellation)
        double r1, t1, r2, t2;
        direct_terms(tau, w, g, g1, g2, k, L.R, L.T, mu0 * (1.0 - kShift), &r1, &t1);
        direct_terms(tau, w, g, g1, g2, k, L.R, L.T, mu0 * (1.0 + kShift), &r2, &t2);
        L.Rdir = 0.5 * (r1 + r2);
        L.Tdir = 0.5 * (t1 + t2);
    } else {
        direct_terms(tau, w, g, g1, g2, k, L.R, L.T, mu0, &L.Rdir, &L.Tdir);
    }
    L.Tb = exp(-tau / mu0);
    return L;
}

// Adding method per column.  Up sweep from the surface: rb = diffuse albedo
// of everything below a level, q = upward diffuse flux there produced by the
// direct beam below it; both are parked in flux_up / flux_dn_dif.  Down
// sweep: diffuse downward flux from multiple reflection between a layer and
// what lies below it, then up = rb * down + q overwrites the scratch.
__global__ void two_stream_kernel(int ncols, int nlay, const double* __restrict__ tau,
                                  const double* __restrict__ ssa, const double* __restrict__ asy,
                                  const double* __restrict__ albedo, double mu0, const double* __restrict__ flux_toa,
                                  double* __restrict__ S, double* __restrict__ D, double* __restrict__ U, int tod,
                                  double* __restrict__ tod_flux, float* __restrict__ tod_fd) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    const size_t lo = (size_t)c * nlay;
    const size_t vo = (size_t)c * (nlay + 1);
    double s = (flux_toa ? flux_toa[c] : 1.0) * mu0;
    S[vo] = s;
    for (int l = 0; l < nlay; ++l) {
        s *= exp(-tau[lo + l] / mu0);
        S[vo + l + 1] = s;
    }
    double rb = albedo[c];
    double q = rb * S[vo + nlay];
    U[vo + nlay] = rb;
    D[vo + nlay] = q;
    for (int l = nlay - 1; l >= 0; --l) {
        const LayerRT L = layer_rt(tau[lo + l], ssa[lo + l], asy[lo + l], mu0);
        const double m = 1.0 / (1.0 - L.R * rb);
        const double sl = S[vo + l];
        q = L.Rdir * sl + L.T * (q + rb * L.Tdir * sl) * m;
        rb = L.R + L.T * L.T * rb * m;
        U[vo + l] = rb;
        D[vo + l] = q;
    }
    // top of the atmosphere: no diffuse light comes down
    U[vo] = D[vo];
    D[vo] = 0.0;
    double dn = 0.0;
    for (int l = 0; l < nlay; ++l) {
        const LayerRT L = layer_rt(tau[lo + l], ssa[lo + l], asy[lo + l], mu0);
        const double rbn = U[vo + l + 1];
        const double qn = D[vo + l + 1];
        dn = (L.T * dn + L.Tdir * S[vo + l] + L.R * qn) / (1.0 - L.R * rbn);
        D[vo + l + 1] = dn;
        U[vo + l + 1] = rbn * dn + qn;
    }
    const double tot = S[vo + tod] + D[vo + tod];
    if (tod_flux) tod_flux[c] = tot;
    if (tod_fd) tod_fd[c] = tot > 0.0 ? (float)(D[vo + tod] / tot) : 0.0f;
}

}  // namespace

extern "C" {

rt3d_status rt3d_two_stream(int32_t n_cols, int32_t nlay, const double* tau, const double* ssa, const double* g,
                            const double* albedo, double mu0, const double* flux_toa, double* flux_dir,
                            double* flux_dn_dif, double* flux_up, int32_t tod_level, double* tod_flux,
                            float* tod_diffuse_fraction, void* stream) {
    if (n_cols < 1 || nlay < 1 || !tau || !ssa || !g || !albedo || !flux_dir || !flux_dn_dif || !flux_up)
        return RT3D_EINVAL;
    if (!(mu0 > 0.0 && mu0 <= 1.0)) return RT3D_EINVAL;
    if (tod_level < 0 || tod_level > nlay) return RT3D_EINVAL;
    hipLaunchKernelGGL(two_stream_kernel, dim3((n_cols + 63) / 64), dim3(64), 0, (hipStream_t)stream, n_cols, nlay,
                       tau, ssa, g, albedo, mu0, flux_toa, flux_dir, flux_dn_dif, flux_up, tod_level, tod_flux,
                       tod_diffuse_fraction);
    return hipGetLastError() == hipSuccess ? RT3D_OK : RT3D_EDEVICE;
}

}  // extern "C"
