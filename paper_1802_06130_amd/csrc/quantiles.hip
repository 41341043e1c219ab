// Equal-population thresholds of a feature over all training pixels: the k/q quantiles
// (k = 1 .. q-1) with linear interpolation between order statistics. The values are sorted on
// the device with hipCUB's radix sort; only the 2(q-1) neighbouring order statistics are copied
// back, and the interpolation is done on the host.

#include <hipcub/hipcub.hpp>

#include "mdn_internal.h"

namespace mdn {

size_t quantile_ws_bytes(int64_t n) {
    size_t tmp = 0;
    double* k = nullptr;
    hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, k, k, (int)n);
    return (tmp + 255) / 256 * 256 + ((size_t)n * 8 + 255) / 256 * 256;
}

mdn_status quantiles(const double* values, int64_t n, int q, double* out_host, void* ws, size_t ws_bytes,
                     hipStream_t st) {
    size_t tmp = 0;
    double* k = nullptr;
    hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, k, k, (int)n);
    const size_t tmp_al = (tmp + 255) / 256 * 256;
    double* sorted = reinterpret_cast<double*>(static_cast<char*>(ws) + tmp_al);
    if (hipcub::DeviceRadixSort::SortKeys(ws, tmp, values, sorted, (int)n, 0, 64, st) != hipSuccess)
        return fail(MDN_EDEVICE, "quantiles: radix sort failed");
    for (int j = 1; j < q; ++j) {
        const double pos = (double)(n - 1) * (double)j / (double)q;
        int64_t lo = (int64_t)pos;
        if (lo > n - 1) lo = n - 1;
        const int64_t hi = lo + 1 < n ? lo + 1 : lo;
        double v[2];
        if (hipMemcpyAsync(&v[0], sorted + lo, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&v[1], sorted + hi, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(MDN_EDEVICE, "quantiles: copy failed");
        const double t = pos - (double)lo;
        out_host[j - 1] = v[0] + (v[1] - v[0]) * t;
    }
    (void)ws_bytes;
    return MDN_OK;
}

}  // namespace mdn
