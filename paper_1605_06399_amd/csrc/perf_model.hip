// Performance model of the model-guided auto-tuner (Section 4: the auto-tuner times a random
// sample of parameter configurations, fits an artificial neural network that predicts the
// execution time of a configuration, predicts every configuration, and times the ones with
// the best predictions).
//
// The network: d standardised inputs, one hidden layer of tanh units, one linear output that
// predicts the standardised logarithm of the time.  Full-batch Adam on the squared error with
// a small L2 penalty, weights initialised from a SplitMix64 stream of the given seed, so a fit
// is deterministic.  Host code only; nothing here touches the GPU.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "icl_internal.hpp"

namespace icl {

namespace {

uint64_t splitmix_next(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform_pm1(uint64_t& s) { return ((splitmix_next(s) >> 11) * 0x1.0p-53) * 2.0 - 1.0; }

}  // namespace

bool PerfModel::fit(const std::vector<std::vector<double>>& X, const std::vector<double>& y, int hidden, int iters,
                    uint64_t seed) {
    const int n = (int)X.size();
    if (n < 2 || (int)y.size() != n || hidden < 1 || iters < 1) return false;
    d = (int)X[0].size();
    for (const auto& row : X)
        if ((int)row.size() != d) return false;
    h = hidden;
    // standardise inputs (constant columns get unit scale) and the target
    mu.assign(d, 0.0);
    sd.assign(d, 0.0);
    for (const auto& row : X)
        for (int j = 0; j < d; ++j) mu[j] += row[j] / n;
    for (const auto& row : X)
        for (int j = 0; j < d; ++j) sd[j] += (row[j] - mu[j]) * (row[j] - mu[j]) / n;
    for (int j = 0; j < d; ++j) sd[j] = sd[j] > 1e-12 ? std::sqrt(sd[j]) : 1.0;
    ymu = 0.0;
    for (double v : y) ymu += v / n;
    double yv = 0.0;
    for (double v : y) yv += (v - ymu) * (v - ymu) / n;
    ysd = yv > 1e-24 ? std::sqrt(yv) : 1.0;
    std::vector<std::vector<double>> Z(n, std::vector<double>(d));
    std::vector<double> t(n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) Z[i][j] = (X[i][j] - mu[j]) / sd[j];
        t[i] = (y[i] - ymu) / ysd;
    }
    // parameters: w1[h][d], b1[h], w2[h], b2 packed in one vector
    const int np = h * d + h + h + 1;
    p.assign(np, 0.0);
    uint64_t s = seed;
    const double a1 = 1.0 / std::sqrt((double)d), a2 = 1.0 / std::sqrt((double)h);
    for (int k = 0; k < h * d; ++k) p[k] = a1 * uniform_pm1(s);
    for (int k = 0; k < h; ++k) p[h * d + h + k] = a2 * uniform_pm1(s);
    std::vector<double> g(np), m1(np, 0.0), m2(np, 0.0), hid(h);
    const double lr = 0.01, b1r = 0.9, b2r = 0.999, eps = 1e-8, l2 = 1e-4;
    for (int it = 1; it <= iters; ++it) {
        std::fill(g.begin(), g.end(), 0.0);
        for (int i = 0; i < n; ++i) {
            double out = p[np - 1];
            for (int u = 0; u < h; ++u) {
                double a = p[h * d + u];
                for (int j = 0; j < d; ++j) a += p[u * d + j] * Z[i][j];
                hid[u] = std::tanh(a);
                out += p[h * d + h + u] * hid[u];
            }
            const double e = 2.0 * (out - t[i]) / n;   // d(mean squared error)/d(out)
            g[np - 1] += e;
            for (int u = 0; u < h; ++u) {
                g[h * d + h + u] += e * hid[u];
                const double da = e * p[h * d + h + u] * (1.0 - hid[u] * hid[u]);
                g[h * d + u] += da;
                for (int j = 0; j < d; ++j) g[u * d + j] += da * Z[i][j];
            }
        }
        for (int k = 0; k < np - 1; ++k) g[k] += l2 * p[k];
        const double c1 = 1.0 - std::pow(b1r, it), c2 = 1.0 - std::pow(b2r, it);
        for (int k = 0; k < np; ++k) {
            m1[k] = b1r * m1[k] + (1.0 - b1r) * g[k];
            m2[k] = b2r * m2[k] + (1.0 - b2r) * g[k] * g[k];
            p[k] -= lr * (m1[k] / c1) / (std::sqrt(m2[k] / c2) + eps);
        }
    }
    return true;
}

double PerfModel::predict(const std::vector<double>& x) const {
    const int np = (int)p.size();
    double out = p[np - 1];
    for (int u = 0; u < h; ++u) {
        double a = p[h * d + u];
        for (int j = 0; j < d; ++j) a += p[u * d + j] * (x[j] - mu[j]) / sd[j];
        out += p[h * d + h + u] * std::tanh(a);
    }
    return out * ysd + ymu;
}

// Numeric description of a variant from its name: the leading token is the family
// (one-hot); each later token such as t32, c1, o2, p8x2 gives log2 of its numbers under its
// letter key (p8x2: keys p and p.y).  Tokens without digits join the family name.
void variant_features(const std::vector<std::string>& names, std::vector<std::vector<double>>& F) {
    struct Parsed {
        std::string family;
        std::vector<std::pair<std::string, double>> kv;
    };
    std::vector<Parsed> ps;
    std::vector<std::string> families, keys;
    for (const auto& nm : names) {
        Parsed q;
        size_t pos = 0;
        bool first = true;
        while (pos <= nm.size()) {
            size_t e = nm.find('_', pos);
            if (e == std::string::npos) e = nm.size();
            const std::string tok = nm.substr(pos, e - pos);
            size_t dpos = tok.find_first_of("0123456789");
            const bool param = !first && dpos != std::string::npos && dpos > 0 &&
                               tok.find_first_not_of("0123456789x", dpos) == std::string::npos;
            if (!param) {
                q.family += (q.family.empty() ? "" : "_") + tok;
            } else {
                const std::string key = tok.substr(0, dpos);
                const std::string nums = tok.substr(dpos);
                const size_t xp = nums.find('x');
                const double a = std::atof(nums.substr(0, xp).c_str());
                q.kv.push_back({key, std::log2(std::max(a, 1.0))});
                if (xp != std::string::npos)
                    q.kv.push_back({key + ".y", std::log2(std::max(std::atof(nums.substr(xp + 1).c_str()), 1.0))});
            }
            first = false;
            pos = e + 1;
        }
        if (std::find(families.begin(), families.end(), q.family) == families.end()) families.push_back(q.family);
        for (const auto& kv : q.kv)
            if (std::find(keys.begin(), keys.end(), kv.first) == keys.end()) keys.push_back(kv.first);
        ps.push_back(q);
    }
    F.assign(names.size(), std::vector<double>(families.size() + keys.size(), 0.0));
    for (size_t i = 0; i < ps.size(); ++i) {
        const size_t f = std::find(families.begin(), families.end(), ps[i].family) - families.begin();
        F[i][f] = 1.0;
        for (const auto& kv : ps[i].kv) {
            const size_t k = std::find(keys.begin(), keys.end(), kv.first) - keys.begin();
            F[i][families.size() + k] = kv.second;
        }
    }
}

}  // namespace icl

using namespace icl;

extern "C" icl_status icl_perf_model_fit_predict(const double* X, const double* y, int n, int d, const double* Xq,
                                                 int nq, double* yq, int hidden, int iters,
                                                 unsigned long long seed) {
    if (!X || !y || n < 2 || d < 1 || nq < 0 || (nq > 0 && (!Xq || !yq)) || hidden < 1 || hidden > 256 ||
        iters < 1 || iters > 1000000)
        return ICL_ERR_INVALID_VALUE;
    std::vector<std::vector<double>> XX(n, std::vector<double>(d));
    std::vector<double> yy(y, y + n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j) XX[i][j] = X[(size_t)i * d + j];
    PerfModel m;
    if (!m.fit(XX, yy, hidden, iters, seed)) return ICL_ERR_INVALID_VALUE;
    std::vector<double> row(d);
    for (int i = 0; i < nq; ++i) {
        for (int j = 0; j < d; ++j) row[j] = Xq[(size_t)i * d + j];
        yq[i] = m.predict(row);
    }
    return ICL_OK;
}
