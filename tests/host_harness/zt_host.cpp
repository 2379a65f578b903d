// Host build of the library's coefficient math (the same source the device
// setup kernels include), so that tests can compare it with the oracle on a
// machine without a GPU.  Test infrastructure only.
#include <cmath>
#include <cstdint>
using std::fmin;
using std::fmax;

namespace tdbem {
struct GeoDev {
    const double *xyz; const int *tri; const double *area; const double *nrm; const double *qpt;
    const int *etri; const int *efree; const double *elen;
    double cdt, dt, eps, mu, theta, zeta, eta;
    double kd;
};
#define TD_HD static inline
#define TD_CONST static const
#include "../../paper_2303_05006_amd/csrc/zt_integrals.inl"
}  // namespace tdbem

using tdbem::GeoDev;

static GeoDev mk(const double *xyz, const int *tri, const double *area, const double *nrm, const double *qpt,
                 const int *etri, const int *efree, const double *elen, const double *par) {
    return GeoDev{xyz, tri, area, nrm, qpt, etri, efree, elen, par[0], par[1], par[2], par[3], par[4], par[5], par[6],
                  par[7]};
}

extern "C" {
// par = cdt, dt, eps, mu, theta, zeta, eta, kd
void zt_host(const double *xyz, const int *tri, const double *area, const double *nrm, const double *qpt,
             const int *etri, const int *efree, const double *elen, const double *par,
             long npairs, const int *pi, const int *pj, int G, double *out, int *lo, int *hi) {
    GeoDev g = mk(xyz, tri, area, nrm, qpt, etri, efree, elen, par);
#pragma omp parallel for schedule(dynamic, 16)
    for (long p = 0; p < npairs; ++p) {
        int a, b;
        tdbem::pair_lag_range(g, pi[p], pj[p], a, b);
        lo[p] = a;
        hi[p] = b;
        for (int k = 0; k < G; ++k) out[(size_t)p * G + k] = 0.0;
        for (int k = a; k <= b && k < G; ++k) out[(size_t)p * G + k] = tdbem::zt_value(g, pi[p], pj[p], k);
    }
}
void vinc_host(const double *xyz, const int *tri, const double *area, const double *nrm, const double *qpt,
               const int *etri, const int *efree, const double *elen, const double *par,
               int ne, const double *pulse, double t, double *out) {
    GeoDev g = mk(xyz, tri, area, nrm, qpt, etri, efree, elen, par);
    for (int p = 0; p < ne; ++p) out[p] = tdbem::vinc_value(g, p, pulse, t);
}
}
