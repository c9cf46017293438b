// The cost model of Sec. 5.3 and the fanout it prefers.
//
// A range query descends L = ceil(log_F n) layers; at layer i the objects
// not yet pruned number about F^i p^i, where p bounds from below the
// probability that one pivot fails to prune an object.  With X, Y the
// distances of an object and of the query to a pivot (independent, equally
// distributed, variance sigma^2), X - Y has mean 0 and variance 2 sigma^2,
// and Chebyshev's inequality gives P(|X - Y| <= r) >= 1 - 2 sigma^2 / r^2
// (Eq. 3).  Each layer costs ceil(S_i / C) parallel rounds of a sort of
// log^2 work over the layer's intermediate results (Eq. 2), which gives
//   cost(F) = sum_{i=1..L} i^2 ceil(F^i p^i / C) log2(F)^2.
// Readings: p is clamped to [0, 1] (the bound is vacuous when r^2 < 2
// sigma^2), and a layer costs at least one round (ceil of a positive count;
// the root path is always visited).
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "gts_internal.h"

namespace gts {
namespace {

double model_cost(int64_t n, int F, double sigma2, double r, double C)
{
    if (n < 1 || F < 2 || C <= 0.0) return NAN;
    double p = r > 0.0 ? 1.0 - 2.0 * sigma2 / (r * r) : 0.0;
    p = std::min(1.0, std::max(0.0, p));
    int L = 0;
    for (double cap = 1.0; cap < (double)n; cap *= F) L++;
    L = std::max(L, 1);
    const double lg = std::log2((double)F);
    double cost = 0.0, layer = 1.0;
    for (int i = 1; i <= L; i++) {
        layer *= F * p;
        const double rounds = std::max(1.0, std::ceil(layer / C));
        cost += (double)i * i * rounds * lg * lg;
    }
    return cost;
}

// Levenshtein distance by the two-row table (the sample's distances only)
int edit_distance(const uint8_t *a, int la, const uint8_t *b, int lb)
{
    std::vector<int> prev(lb + 1), cur(lb + 1);
    for (int j = 0; j <= lb; j++) prev[j] = j;
    for (int i = 1; i <= la; i++) {
        cur[0] = i;
        for (int j = 1; j <= lb; j++)
            cur[j] = std::min({prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0)});
        std::swap(prev, cur);
    }
    return prev[lb];
}

}  // namespace
}  // namespace gts

using namespace gts;

extern "C" {

double gts_cost_model(int64_t n, int32_t fanout, double sigma2, double radius, double concurrency)
{
    return model_cost(n, fanout, sigma2, radius, concurrency);
}

gts_status gts_choose_fanout(const gts_objects *objs, int32_t metric, float radius, double concurrency,
                             int32_t *fanout, double *costs)
{
    return run_guarded([&] {
        GTS_CHECK(objs != nullptr && fanout != nullptr, GTS_EINVAL, "null argument");
        GTS_CHECK(metric == GTS_L2_F32 || metric == GTS_EDIT_U8 || metric == GTS_COSINE_F32, GTS_EINVAL,
                  "unknown metric");
        GTS_CHECK(std::isfinite(radius) && radius >= 0.f, GTS_EINVAL, "radius must be finite and >= 0");
        GTS_CHECK(objs->n >= 2, GTS_EINVAL, "the sample needs at least two objects");
        const bool angular = metric == GTS_COSINE_F32;
        const int32_t m = angular ? GTS_L2_F32 : metric;
        HostObjects h;
        read_objects(objs, m, m == GTS_L2_F32 ? objs->dim : 0, kMaxStrlen, &h, angular);
        // sigma^2: distances of a seeded sample of objects to one sample pivot
        const int64_t n = h.count();
        const int64_t take = std::min<int64_t>(n - 1, 2048);
        uint64_t s = 0x2404009661ULL;
        auto next = [&]() {
            s += 0x9e3779b97f4a7c15ULL;
            uint64_t z = s;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
            return z ^ (z >> 31);
        };
        const int64_t piv = (int64_t)(next() % (uint64_t)n);
        double sum = 0.0, sum2 = 0.0;
        for (int64_t t = 0; t < take; t++) {
            int64_t o = (int64_t)(next() % (uint64_t)(n - 1));
            if (o >= piv) o++;
            double d;
            if (m == GTS_L2_F32) {
                double acc = 0.0;
                for (int j = 0; j < h.dim; j++) {
                    const double df = (double)h.vecs[(size_t)o * h.dim + j] - h.vecs[(size_t)piv * h.dim + j];
                    acc += df * df;
                }
                d = std::sqrt(acc);
            } else {
                d = edit_distance(h.chars.data() + h.offsets[o], (int)(h.offsets[o + 1] - h.offsets[o]),
                                  h.chars.data() + h.offsets[piv], (int)(h.offsets[piv + 1] - h.offsets[piv]));
            }
            sum += d;
            sum2 += d * d;
        }
        const double mean = sum / (double)take;
        const double sigma2 = std::max(0.0, sum2 / (double)take - mean * mean);
        double C = concurrency;
        if (C <= 0.0) {
            int dev = 0, cus = 256;
            GTS_HIP(hipGetDevice(&dev));
            GTS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            C = (double)cus * 2048.0;   // resident threads of the device
        }
        // the chord of the angular radius (the index is L2 on unit vectors)
        const double r = angular ? 2.0 * std::sin(std::min((double)radius, M_PI) / 2.0) : (double)radius;
        int best = 2;
        double best_cost = INFINITY;
        for (int F = 2; F <= 64; F++) {
            const double c = model_cost(n, F, sigma2, r, C);
            if (costs) costs[F - 2] = c;
            if (c < best_cost) {
                best_cost = c;
                best = F;
            }
        }
        *fanout = best;
    });
}

}  // extern "C"
