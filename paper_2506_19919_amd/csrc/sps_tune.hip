// Launch choices that never change a result (tile order, XCD placement, iterations per
// launch, graph replay) and their autotuner: each candidate is timed with HIP events on the
// caller's stream and inputs, the fastest is kept in the context and, if SPS_AUTOTUNE_CACHE
// names a file, recorded there for later runs (a JSON object, one entry per line).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "sps_internal.h"

namespace sps {
namespace {

bool launch_valid(const sps_launch_cfg &l) {
    return l.exact_order >= 0 && l.exact_order <= 3 && (l.exact_xcd == 0 || l.exact_xcd == 1) &&
           l.hmc_block_iters >= 1 && l.hmc_block_iters <= 1000 && l.nuts_block_iters >= 1 &&
           l.nuts_block_iters <= 1000 && (l.hmcx_graph == 0 || l.hmcx_graph == 1) &&
           (l.exact_ring == 0 || l.exact_ring == 1);
}

// ---- the cache file: {"key": {"name": value, ...}, ...}, one entry per line
typedef std::map<std::string, std::map<std::string, double>> Cache;

std::string cache_path() {
    const char *p = std::getenv("SPS_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// reads the entries this file's writer produced (other content is skipped)
Cache cache_read(const std::string &path) {
    Cache out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t k0 = line.find('"');
        if (k0 == std::string::npos) continue;
        const size_t k1 = line.find('"', k0 + 1), b0 = line.find('{', k1 == std::string::npos ? 0 : k1);
        if (k1 == std::string::npos || b0 == std::string::npos) continue;
        const std::string key = line.substr(k0 + 1, k1 - k0 - 1);
        std::map<std::string, double> vals;
        size_t at = b0 + 1;
        for (;;) {
            const size_t n0 = line.find('"', at);
            if (n0 == std::string::npos) break;
            const size_t n1 = line.find('"', n0 + 1), colon = line.find(':', n1 == std::string::npos ? n0 : n1);
            if (n1 == std::string::npos || colon == std::string::npos) break;
            char *end = nullptr;
            const double v = std::strtod(line.c_str() + colon + 1, &end);
            if (end == line.c_str() + colon + 1) break;
            vals[line.substr(n0 + 1, n1 - n0 - 1)] = v;
            at = (size_t)(end - line.c_str());
        }
        if (!vals.empty()) out[key] = vals;
    }
    return out;
}

void cache_write(const std::string &path, const Cache &c) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;
        f << "{\n";
        size_t i = 0;
        for (const auto &e : c) {
            f << "  \"" << e.first << "\": {";
            size_t j = 0;
            for (const auto &v : e.second) {
                char buf[64];
                std::snprintf(buf, sizeof buf, "%.9g", v.second);
                f << "\"" << v.first << "\": " << buf << (++j < e.second.size() ? ", " : "");
            }
            f << "}" << (++i < c.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

std::string device_key(int device) {
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::ostringstream o;
    o << p.gcnArchName << "/" << p.multiProcessorCount << "cu";
    std::string s = o.str();
    for (char &ch : s)
        if (ch == '"' || ch == '\\' || ch == ':') ch = '_';
    return s;
}

// median of reps timings (ms) of run() on stream s, after one untimed call
template <class F>
int time_median(hipStream_t s, int reps, F run, float *ms) {
    hipEvent_t e0, e1;
    SPS_HIP(hipEventCreate(&e0));
    SPS_HIP(hipEventCreate(&e1));
    int rc = run();
    std::vector<float> t;
    for (int r = 0; r < reps && !rc; ++r) {
        (void)hipEventRecord(e0, s);
        rc = run();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float v = 0.0f;
        (void)hipEventElapsedTime(&v, e0, e1);
        t.push_back(v);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return SPS_OK;
}

// picks the fastest of the candidates (each applied to a copy of the context's launch
// choices by set), caching the result under key; *ms_out: its time, 0 if cached
template <class Set, class Run>
int tune(sps_ctx *c, hipStream_t s, const std::string &key, const std::vector<std::map<std::string, double>> &cands,
         Set set, Run run, sps_launch_cfg *chosen, float *ms_out) {
    const std::string path = cache_path();
    Cache cache;
    if (!path.empty()) {
        cache = cache_read(path);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            sps_launch_cfg l = c->launch;
            set(l, it->second);
            if (launch_valid(l)) {
                c->launch = l;
                if (chosen) *chosen = l;
                if (ms_out) *ms_out = 0.0f;
                return SPS_OK;
            }
        }
    }
    const sps_launch_cfg base = c->launch;
    float best = 0.0f;
    int ib = -1;
    for (size_t i = 0; i < cands.size(); ++i) {
        sps_launch_cfg l = base;
        set(l, cands[i]);
        c->launch = l;
        float ms = 0.0f;
        const int rc = time_median(s, 3, run, &ms);
        if (rc) {
            c->launch = base;
            return rc;
        }
        if (ib < 0 || ms < best) {
            best = ms;
            ib = (int)i;
        }
    }
    sps_launch_cfg l = base;
    set(l, cands[ib]);
    c->launch = l;
    if (chosen) *chosen = l;
    if (ms_out) *ms_out = best;
    if (!path.empty()) {
        auto entry = cands[ib];
        entry["ms"] = best;
        cache[key] = entry;
        cache_write(path, cache);
    }
    return SPS_OK;
}

}  // namespace
}  // namespace sps

using namespace sps;

extern "C" {

int sps_get_launch(sps_ctx *c, sps_launch_cfg *out) {
    if (!c || !out) return set_error(SPS_E_INVAL, "sps_get_launch: null argument");
    *out = c->launch;
    return SPS_OK;
}

int sps_set_launch(sps_ctx *c, const sps_launch_cfg *l) {
    if (!c || !l) return set_error(SPS_E_INVAL, "sps_set_launch: null argument");
    if (!launch_valid(*l)) return set_error(SPS_E_INVAL, "sps_set_launch: a launch choice is out of range");
    c->launch = *l;
    return SPS_OK;
}

int sps_autotune_exact(sps_ctx *c, void *stream, int n_gal, int sfh, int prec, const float *params, const float *z,
                       const float *obs, const float *sigma, const uint8_t *band_mask, sps_launch_cfg *chosen,
                       float *timed_ms) {
    if (!c) return set_error(SPS_E_INVAL, "null context");
    if (prec != SPS_F32 && prec != SPS_BF16X) return set_error(SPS_E_INVAL, "the exact-path tuner takes SPS_F32 or SPS_BF16X");
    if (n_gal < 1 || !params || !z) return set_error(SPS_E_INVAL, "sps_autotune_exact: need n_gal >= 1, params and z");
    SPS_HIP(hipSetDevice(c->device));
    const bool lik = obs && sigma && band_mask;
    float *logl = nullptr, *grad = nullptr, *mags = nullptr;
    if (lik) {
        SPS_HIP(hipMalloc(&logl, (size_t)n_gal * sizeof(float)));
        SPS_HIP(hipMalloc(&grad, (size_t)n_gal * SPS_NPARAM * sizeof(float)));
    } else {
        SPS_HIP(hipMalloc(&mags, (size_t)n_gal * c->n_band * sizeof(float)));
    }
    const hipStream_t s = (hipStream_t)stream;
    std::ostringstream key;
    key << "exact|" << device_key(c->device) << "|n=" << n_gal << "|prec=" << prec << "|nw=" << c->n_wave
        << "|nb=" << c->n_band << "|grad=" << (lik ? 1 : 0);
    std::vector<std::map<std::string, double>> cands;
    for (int rg = 0; rg <= (prec == SPS_BF16X ? 1 : 0); ++rg)
        for (int o = 0; o <= 3; ++o)
            for (int x = 1; x >= 0; --x)
                cands.push_back({{"exact_order", (double)o}, {"exact_xcd", (double)x}, {"exact_ring", (double)rg}});
    auto set = [](sps_launch_cfg &l, const std::map<std::string, double> &v) {
        auto o = v.find("exact_order"), x = v.find("exact_xcd"), r = v.find("exact_ring");
        if (o != v.end()) l.exact_order = (int)o->second;
        if (x != v.end()) l.exact_xcd = (int)x->second;
        if (r != v.end()) l.exact_ring = (int)r->second;
    };
    auto run = [&]() {
        return lik ? sps_loglike_grad(c, stream, n_gal, sfh, SPS_PATH_EXACT, prec, params, z, obs, sigma, band_mask,
                                      logl, grad)
                   : sps_phot_exact(c, stream, n_gal, sfh, prec, params, z, mags);
    };
    const int rc = tune(c, s, key.str(), cands, set, run, chosen, timed_ms);
    (void)hipStreamSynchronize(s);
    (void)hipFree(logl);
    (void)hipFree(grad);
    (void)hipFree(mags);
    return rc;
}

int sps_autotune_hmc(sps_ctx *c, void *stream, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
                     const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                     const float *prior, const float *theta0, sps_launch_cfg *chosen, float *timed_ms) {
    if (!c || !cfg) return set_error(SPS_E_INVAL, "null argument");
    if (n_gal < 1 || cfg->n_chain < 1) return set_error(SPS_E_INVAL, "sps_autotune_hmc: need n_gal, n_chain >= 1");
    SPS_HIP(hipSetDevice(c->device));
    const bool exact = cfg->path == SPS_PATH_EXACT;
    const int nit = cfg->n_warmup + cfg->n_sample;
    const int trial = std::min(nit, exact ? 10 : 50);
    sps_hmc_cfg t = *cfg;
    t.it_begin = 0;
    t.it_end = trial;
    const size_t fb = (size_t)n_gal * (3 * SPS_NPARAM + 1 + cfg->n_chain * (1 + SPS_NPARAM)) * sizeof(float);
    void *state = nullptr;
    float *sum = nullptr;
    SPS_HIP(hipMalloc(&state, sps_hmc_state_bytes(n_gal, cfg->n_chain)));
    SPS_HIP(hipMalloc(&sum, fb));
    float *pm = sum, *ps = pm + (size_t)SPS_NPARAM * n_gal, *rh = ps + (size_t)SPS_NPARAM * n_gal;
    float *acc = rh + (size_t)SPS_NPARAM * n_gal, *stp = acc + n_gal, *im = stp + (size_t)cfg->n_chain * n_gal;
    const hipStream_t s = (hipStream_t)stream;
    std::ostringstream key;
    key << (exact ? "hmc_exact|" : "hmc|") << device_key(c->device) << "|n=" << n_gal << "|C=" << cfg->n_chain
        << "|L=" << cfg->n_leapfrog << "|nb=" << c->n_band << "|nw=" << c->n_wave << (exact ? "|prec=" : "")
        << (exact ? std::to_string(cfg->prec) : std::string());
    std::vector<std::map<std::string, double>> cands;
    if (exact) {
        cands = {{{"hmcx_graph", 1.0}}, {{"hmcx_graph", 0.0}}};
    } else {
        for (int b : {5, 10, 25, 50}) cands.push_back({{"hmc_block_iters", (double)b}});
    }
    auto set = [](sps_launch_cfg &l, const std::map<std::string, double> &v) {
        auto g = v.find("hmcx_graph"), b = v.find("hmc_block_iters");
        if (g != v.end()) l.hmcx_graph = (int)g->second;
        if (b != v.end()) l.hmc_block_iters = (int)b->second;
    };
    auto run = [&]() {
        return sps_hmc_run(c, stream, &t, n_gal, sfh, z, obs, sigma, band_mask, bounds, prior, theta0, nullptr, pm, ps,
                           rh, acc, stp, im, state);
    };
    const int rc = tune(c, s, key.str(), cands, set, run, chosen, timed_ms);
    (void)hipStreamSynchronize(s);
    (void)hipFree(state);
    (void)hipFree(sum);
    return rc;
}

}  // extern "C"
