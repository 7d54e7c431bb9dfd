// layers.hip -- the method of layers (Sec. 5) in host code: which pairs of
// half-layers of the unstable and stable manifold meshes a connection search
// has to examine, and which s-columns of a mesh form one half-layer
// (Sec. 6.2: a half-layer of a mesh stored column by column is a contiguous
// range of columns).
#include <math.h>

#include "ms_internal.hpp"

extern "C" int layer_pairs(int32_t n_layers, layer_pair_t *out, int32_t cap, int32_t *n_out)
{
    if (n_layers < 0 || !n_out || cap < 0 || (cap > 0 && !out)) return ms::fail(MS_E_ARG, "layer_pairs: bad argument");
    const int64_t n = 8 * (int64_t)n_layers;
    if (n > 0x7fffffff) return ms::fail(MS_E_ARG, "layer_pairs: too many layers");
    *n_out = (int32_t)n;
    if (n > cap) return ms::fail(MS_E_CAPACITY, "layer_pairs: cap below 8 * n_layers");
    int32_t k = 0;
    for (int32_t layer = 1; layer <= n_layers; ++layer)
        for (int32_t a = 0; a < 2; ++a)                 // U_n^+, then U_n^-
            for (int32_t m = 0; m < 2; ++m)             // S_n, then S_{n-1}
                for (int32_t b = 0; b < 2; ++b) {       // S^+, then S^-
                    layer_pair_t &p = out[k++];
                    p.u_layer = layer;
                    p.u_sign = a ? -1 : 1;
                    p.s_layer = layer - m;
                    p.s_sign = b ? -1 : 1;
                }
    return MS_OK;
}

extern "C" int half_layer_bounds(double D, double lambda, int32_t stable, int32_t layer, double *lo, double *hi)
{
    if (!lo || !hi || !(D > 0.0) || !isfinite(D) || !(lambda > 0.0) || !isfinite(lambda) || lambda == 1.0)
        return ms::fail(MS_E_ARG, "half_layer_bounds: need D > 0, lambda > 0, lambda != 1, finite");
    const double b0 = stable ? D / pow(lambda, (double)(layer - 1)) : D * pow(lambda, (double)(layer - 1));
    const double b1 = stable ? D / pow(lambda, (double)layer) : D * pow(lambda, (double)layer);
    if (!isfinite(b0) || !isfinite(b1)) return ms::fail(MS_E_ARG, "half_layer_bounds: bounds overflow");
    *lo = b0 < b1 ? b0 : b1;
    *hi = b0 < b1 ? b1 : b0;
    return MS_OK;
}

extern "C" int half_layer_columns(const double *s_host, int32_t n_s_v, double D, double lambda, int32_t stable,
                                  int32_t layer, int32_t sign, int32_t *k0, int32_t *k1)
{
    if (!s_host || n_s_v < 2 || !k0 || !k1 || (sign != 1 && sign != -1))
        return ms::fail(MS_E_ARG, "half_layer_columns: bad argument");
    for (int32_t k = 1; k < n_s_v; ++k)
        if (!(s_host[k] > s_host[k - 1])) return ms::fail(MS_E_ARG, "half_layer_columns: s must increase strictly");
    double lo, hi;
    int rc = half_layer_bounds(D, lambda, stable, layer, &lo, &hi);
    if (rc) return rc;
    if (sign < 0) {
        const double t = lo;
        lo = -hi;
        hi = -t;
    }
    // the boundary columns must be samples (within a relative 1e-12)
    const double tol = 1e-12 * (fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi));
    int32_t a = -1, b = -1;
    for (int32_t k = 0; k < n_s_v; ++k) {
        if (a < 0 && fabs(s_host[k] - lo) <= tol) a = k;
        if (fabs(s_host[k] - hi) <= tol) b = k;
    }
    if (a < 0 || b < 0 || b <= a)
        return ms::fail(MS_E_ARG, "half_layer_columns: the half-layer's boundaries are not s samples");
    *k0 = a;
    *k1 = b;
    return MS_OK;
}
