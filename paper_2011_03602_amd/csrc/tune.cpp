// Genetic-algorithm tile tuner, in the style of the paper's loop-offload
// search (Sec. 4.2.2): the search space is encoded as bit genes, the initial
// population is random, every individual is built and measured on the real
// device, a gene that cannot be built scores zero (the paper drops loops whose
// directive does not compile), a gene whose results differ from the original
// CPU program beyond a tolerance is given infinite time (the paper's result
// check), fitness comes from the measured time, and selection, crossover,
// mutation and an unchanged copy of the best individuals form the next
// generation for a set number of generations; the best gene wins.
//
// Gene layout (bit 0 first):
//   bits 0-1  vec       00:1 01:2 10:4 11:8 (single grids, k-march only;
//                       not buildable for batches or with OFL_TILE_MARCH_J)
//   bits 2-3  rows      1, 2, 4, 8
//   bits 4-6  kchunk    1, 2, 4, ..., 128 (the short chunks measure best on
//                       MI355X: more work-groups keep more loads in flight)
//   bits 7-11 flags     OFL_TILE_NT_LOADS | OFL_TILE_NT_STORES | OFL_TILE_PREFETCH |
//                       OFL_TILE_MARCH_J | OFL_TILE_XCD_REMAP
//   bits 12-13          occupancy: single grids 0 (no cap), 2, 3, 4 resident
//                       sweep work-groups per CU; batches 0 (one work-group per
//                       item), 2, 4, 8 persistent work-groups per CU
//   bit 14 (batch)      vector width chosen per grid (overrides bits 0-1)
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "abi_util.hpp"
#include "batch.hpp"

namespace ofl {

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();

struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return static_cast<double>(next() >> 11) * 0x1.0p-53; }
};

int gene_bits(bool batch) { return batch ? 15 : 14; }

bool decode(uint32_t gene, bool batch, TileCfg *t) {
    const int v = static_cast<int>(gene & 3u);
    if (v == 3 && (batch || ((gene >> 7) & static_cast<uint32_t>(OFL_TILE_MARCH_J))))
        return false;
    t->vec = 1 << v;
    t->rows = 1 << ((gene >> 2) & 3u);
    t->kchunk = 1 << ((gene >> 4) & 7u);
    t->flags = static_cast<int>((gene >> 7) & 31u);
    const int occ = static_cast<int>((gene >> 12) & 3u);
    t->occupancy = occ == 0 ? 0 : (batch ? (1 << occ) : occ + 1);
    if (batch && ((gene >> 14) & 1u))
        t->vec = 0;
    return true;
}

uint32_t encode(const TileCfg &t, bool batch) {
    // vector code: 1, 2, 4 (also for a batch's per-grid width, vec 0, which
    // sets bit 14 and leaves a buildable code below it), 8
    uint32_t g = t.vec == 1 ? 0u : (t.vec == 2 ? 1u : (t.vec == 8 ? 3u : 2u));
    if (batch && t.vec == 0)
        g |= 1u << 14;
    int r = 0;
    while ((1 << r) < t.rows && r < 3)
        ++r;
    g |= static_cast<uint32_t>(r) << 2;
    int k = 0;
    while ((1 << k) < t.kchunk && k < 7)
        ++k;
    g |= static_cast<uint32_t>(k) << 4;
    g |= static_cast<uint32_t>(t.flags & 31) << 7;
    if (batch) {
        int o = 1;
        while (o < 3 && (1 << o) < t.occupancy)
            ++o;
        g |= static_cast<uint32_t>(t.occupancy == 0 ? 0 : o) << 12;
    } else if (t.occupancy > 0) {
        g |= static_cast<uint32_t>(std::min(std::max(t.occupancy, 2), 4) - 1) << 12;
    }
    return g;
}

// Small ragged check problem in the workload's value ranges (private to the
// tuner's result check).
struct CheckProblem {
    int I, J, K;
    std::vector<float> coef[kNCoef];
    std::vector<float> p0;
};

CheckProblem make_check(int I, int J, int K, uint64_t seed) {
    CheckProblem c{I, J, K, {}, {}};
    const size_t n = static_cast<size_t>(I) * J * K;
    Rng r{seed};
    auto sym = [&](double h) { return static_cast<float>(h * (2.0 * r.uniform() - 1.0)); };
    for (int a = 0; a < kNCoef; ++a)
        c.coef[a].resize(n);
    c.p0.resize(n);
    for (size_t t = 0; t < n; ++t) {
        const float a0 = 1.0f + sym(0.05), a1 = 1.0f + sym(0.05), a2 = 1.0f + sym(0.05);
        c.coef[0][t] = a0;
        c.coef[1][t] = a1;
        c.coef[2][t] = a2;
        c.coef[3][t] = static_cast<float>(1.0 / (2.0 * (static_cast<double>(a0) + a1 + a2)));
        for (int b = 4; b < 7; ++b)
            c.coef[b][t] = sym(0.01);
        for (int b = 7; b < 10; ++b)
            c.coef[b][t] = 1.0f;
        c.coef[11][t] = sym(0.1);
        c.p0[t] = static_cast<float>(r.uniform());
    }
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < J; ++j)
            for (int i = 0; i < I; ++i) {
                const bool in = i > 0 && j > 0 && k > 0 && i < I - 1 && j < J - 1 && k < K - 1;
                c.coef[10][static_cast<size_t>(i) + static_cast<size_t>(I) * (j + static_cast<size_t>(J) * k)] =
                    in ? 1.0f : 0.0f;
            }
    return c;
}

struct HostRun {
    std::vector<float> p, wrk2;
    ofl_grid *g = nullptr;
    ~HostRun() { ofl_grid_destroy(g); }
};

void open_check_grid(const CheckProblem &c, int fmt, int sum_mode, int device, HostRun &h) {
    h.p = c.p0;
    h.wrk2.assign(c.p0.size(), 0.f);
    ofl_grid_desc d{};
    d.I = c.I;
    d.J = c.J;
    d.K = c.K;
    d.coef_format = fmt;
    d.sum_mode = sum_mode;
    d.p = h.p.data();
    d.wrk2 = h.wrk2.data();
    for (int a = 0; a < kNCoef; ++a)
        d.coef[a] = c.coef[a].data();
    d.device = device;
    if (ofl_grid_create(&d, &h.g) != OFL_OK)
        fail(OFL_EINVAL, std::string("tuner check grid: ") + ofl_last_error());
}

// Relative max-norm difference of two iterates over the interior.
double rel_diff(const CheckProblem &c, const std::vector<float> &x, const std::vector<float> &ref) {
    double num = 0.0, den = 0.0;
    for (int k = 1; k < c.K - 1; ++k)
        for (int j = 1; j < c.J - 1; ++j)
            for (int i = 1; i < c.I - 1; ++i) {
                const size_t t = static_cast<size_t>(i) + static_cast<size_t>(c.I) * (j + static_cast<size_t>(c.J) * k);
                num = std::max(num, std::fabs(static_cast<double>(x[t]) - ref[t]));
                den = std::max(den, std::fabs(static_cast<double>(ref[t])));
            }
    return den > 0 ? num / den : num;
}

constexpr int kCheckIters = 3;
constexpr float kCheckOmega = 0.8f;

// Does the tile reproduce the all-CPU nests on small ragged grids?
bool tile_correct(const TileCfg &t, bool batch, int fmt, int sum_mode, int device, double tol) {
    // two i-tiles, two blocks of owned lines and two march chunks, all ragged
    const bool march_j = (t.flags & OFL_TILE_MARCH_J) != 0;
    const int I = kWave * (t.vec > 0 ? t.vec : 4) + 37;
    const int owned = 2 * t.rows + 3;
    const int marched = std::min(t.kchunk, 24) + 7;
    const int J = march_j ? marched : owned;
    const int K = march_j ? owned : marched;
    std::vector<CheckProblem> probs;
    probs.push_back(make_check(I, J, K, 0xC0FFEEULL + static_cast<uint64_t>(I * 131 + J * 7 + K)));
    if (batch) {
        probs.push_back(make_check(std::max(3, I / 3), J + 1, K + 2, 0xBEEFULL + 17));
        probs.push_back(make_check(5, 4, 3, 0xBEEFULL + 29));
    }
    std::vector<std::unique_ptr<HostRun>> gpu(probs.size()), cpu(probs.size());
    std::vector<double> g_gosa(probs.size()), c_gosa(probs.size());
    for (size_t q = 0; q < probs.size(); ++q) {
        gpu[q].reset(new HostRun);
        cpu[q].reset(new HostRun);
        open_check_grid(probs[q], fmt, sum_mode, device, *gpu[q]);
        open_check_grid(probs[q], fmt, sum_mode, device, *cpu[q]);
        if (ofl_set_offload_mask(cpu[q]->g, OFL_MASK_ALL_CPU, OFL_XFER_HOISTED) != OFL_OK ||
            ofl_jacobi_run(cpu[q]->g, kCheckIters, kCheckOmega, &c_gosa[q]) != OFL_OK)
            fail(OFL_EDEVICE, std::string("tuner reference run: ") + ofl_last_error());
    }
    if (batch) {
        std::vector<ofl_grid *> gs;
        for (auto &h : gpu)
            gs.push_back(h->g);
        ofl_batch *b = nullptr;
        const ofl_tile tile = to_tile(t);
        if (ofl_batch_create(gs.data(), static_cast<int>(gs.size()), &tile, &b) != OFL_OK)
            fail(OFL_EDEVICE, std::string("tuner check batch: ") + ofl_last_error());
        const int rc = ofl_batch_run(b, kCheckIters, kCheckOmega, g_gosa.data());
        ofl_batch_destroy(b);
        if (rc != OFL_OK)
            fail(rc, std::string("tuner check batch run: ") + ofl_last_error());
    } else {
        const ofl_tile tile = to_tile(t);
        if (ofl_set_tile(gpu[0]->g, &tile) != OFL_OK ||
            ofl_jacobi_run(gpu[0]->g, kCheckIters, kCheckOmega, &g_gosa[0]) != OFL_OK)
            fail(OFL_EDEVICE, std::string("tuner check run: ") + ofl_last_error());
    }
    for (size_t q = 0; q < probs.size(); ++q) {
        if (!(rel_diff(probs[q], gpu[q]->p, cpu[q]->p) <= tol))
            return false;
        const double gd = std::fabs(g_gosa[q] - c_gosa[q]) / std::max(std::fabs(c_gosa[q]), 1e-300);
        if (!(gd <= 10.0 * tol))
            return false;
    }
    return true;
}

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        hip_check(hipEventCreate(&a), "hipEventCreate");
        hip_check(hipEventCreate(&b), "hipEventCreate");
    }
    ~EventPair() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    double ms() const {
        float t = 0.f;
        hip_check(hipEventElapsedTime(&t, a, b), "hipEventElapsedTime");
        return t;
    }
};

// Time probe_iters iterations with the tile applied (median of repeats).
double time_grid(ofl_grid *g, const TileCfg &t, const ofl_ga_params &ga) {
    g->tile = t;
    grid_run_loop(g, 1, kCheckOmega, 3);  // warm-up
    grid_sync(g);
    EventPair ev;
    std::vector<double> ts;
    for (int r = 0; r < ga.repeats; ++r) {
        hip_check(hipEventRecord(ev.a, g->stream), "hipEventRecord");
        grid_run_loop(g, ga.probe_iters, kCheckOmega, 3);
        hip_check(hipEventRecord(ev.b, g->stream), "hipEventRecord");
        grid_sync(g);
        ts.push_back(ev.ms());
    }
    return median(ts);
}

double time_batch(ofl_batch *b, const TileCfg &t, const ofl_ga_params &ga) {
    if (b->tile.vec != t.vec || b->tile.rows != t.rows || b->tile.kchunk != t.kchunk || b->tile.flags != t.flags ||
        b->tile.occupancy != t.occupancy) {
        const ofl_tile tile = to_tile(t);
        if (ofl_batch_set_tile(b, &tile) != OFL_OK)
            fail(OFL_EINVAL, ofl_last_error());
    }
    batch_build_tables(b);
    batch_launch(b, ga.probe_iters, kCheckOmega);  // warm-up (captures the graph)
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    batch_after_run(b, ga.probe_iters);
    EventPair ev;
    std::vector<double> ts;
    for (int r = 0; r < ga.repeats; ++r) {
        hip_check(hipEventRecord(ev.a, b->stream), "hipEventRecord");
        batch_launch(b, ga.probe_iters, kCheckOmega);
        hip_check(hipEventRecord(ev.b, b->stream), "hipEventRecord");
        hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        batch_after_run(b, ga.probe_iters);
        ts.push_back(ev.ms());
    }
    return median(ts);
}

void check_params(const ofl_ga_params &ga) {
    if (ga.population < 2 || ga.generations < 1 || ga.elite < 0 || ga.elite > ga.population || ga.probe_iters < 1 ||
        ga.repeats < 1 || !(ga.crossover >= 0 && ga.crossover <= 1) || !(ga.mutation >= 0 && ga.mutation <= 1) ||
        !(ga.tolerance > 0))
        fail(OFL_EINVAL, "GA parameters out of range");
}

// The GA proper over genes of `bits` bits; evaluate(gene) returns time in
// ms, +inf for wrong results, or NaN for genes that cannot be built (both
// score zero). Each distinct gene is evaluated once.
struct GaOutcome {
    uint32_t best;
    double best_t;
    int evaluated, rejected;
};

template <class Eval>
GaOutcome ga_search(const ofl_ga_params &ga, int bits, uint32_t seed_gene, Eval &&evaluate) {
    const uint32_t full = bits >= 32 ? 0xffffffffu : ((1u << bits) - 1u);
    Rng rng{ga.seed ^ 0x5EEDULL};
    std::vector<uint32_t> pop(static_cast<size_t>(ga.population));
    for (auto &g : pop)
        g = static_cast<uint32_t>(rng.next()) & full;
    pop[0] = seed_gene & full;  // the current tile competes too
    std::map<uint32_t, double> memo;
    int rejected = 0;
    uint32_t best = pop[0];
    double best_t = kInf;
    auto eval = [&](uint32_t g) {
        auto it = memo.find(g);
        if (it != memo.end())
            return it->second;
        double t;
        {
            TraceRange range("ofl:ga measure gene");
            t = evaluate(g);
        }
        if (!(t > 0.0 && t < kInf)) {  // NaN (not buildable), inf (wrong), or no positive time
            ++rejected;
            t = kInf;
        }
        memo[g] = t;
        return t;
    };
    auto fitness = [](double t) { return (t > 0 && t < kInf) ? 1.0 / std::sqrt(t) : 0.0; };
    for (int gen = 0; gen < ga.generations; ++gen) {
        std::vector<double> f(pop.size());
        for (size_t i = 0; i < pop.size(); ++i) {
            const double t = eval(pop[i]);
            f[i] = fitness(t);
            if (t < best_t) {
                best_t = t;
                best = pop[i];
            }
        }
        if (gen + 1 == ga.generations)
            break;
        std::vector<size_t> order(pop.size());
        for (size_t i = 0; i < order.size(); ++i)
            order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return f[a] > f[b]; });
        std::vector<uint32_t> next;
        for (int e = 0; e < ga.elite; ++e)
            next.push_back(pop[order[static_cast<size_t>(e)]]);
        const double total = std::accumulate(f.begin(), f.end(), 0.0);
        auto pick = [&]() -> uint32_t {
            if (total <= 0)
                return pop[static_cast<size_t>(rng.next() % pop.size())];
            double x = rng.uniform() * total;
            for (size_t i = 0; i < pop.size(); ++i) {
                x -= f[i];
                if (x < 0)
                    return pop[i];
            }
            return pop.back();
        };
        while (static_cast<int>(next.size()) < ga.population) {
            uint32_t a = pick(), b = pick();
            if (rng.uniform() < ga.crossover) {
                const int cut = 1 + static_cast<int>(rng.next() % static_cast<uint64_t>(bits - 1));
                const uint32_t lo = (1u << cut) - 1u;
                const uint32_t ca = (a & lo) | (b & ~lo);
                const uint32_t cb = (b & lo) | (a & ~lo);
                a = ca;
                b = cb;
            }
            for (uint32_t *c : {&a, &b}) {
                for (int bit = 0; bit < bits; ++bit)
                    if (rng.uniform() < ga.mutation)
                        *c ^= 1u << bit;
                if (static_cast<int>(next.size()) < ga.population)
                    next.push_back(*c & full);
            }
        }
        pop.swap(next);
    }
    return GaOutcome{best, best_t, static_cast<int>(memo.size()), rejected};
}

// ---- measurements kept across searches (checkpoint and resume)
//
// One line per measured gene, appended as soon as it is measured:
//   ofl-tune 1 <key> <gene, hex> <ms | inf | nan>
// The key names everything a gene's time depends on besides the gene: the
// grid shapes and formats, summation mode, fusion, row alignment, the GA's
// timing and check parameters, the device and the library's sources. A
// search under the same key takes those times instead of measuring again.

#ifndef OFL_SOURCE_HASH
#define OFL_SOURCE_HASH "unknown"
#endif

std::mutex g_cache_mu;
std::string g_cache_path;  // empty: no file

class TuneCache {
  public:
    TuneCache(const std::string &path, std::string key) : key_(std::move(key)) {
        if (path.empty())
            return;
        std::ifstream in(path);  // a missing file is an empty cache
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string tag, ver, k, gene_hex, t;
            if (!(ls >> tag >> ver >> k >> gene_hex >> t) || tag != "ofl-tune" || ver != "1" || k != key_)
                continue;
            char *end = nullptr;
            const unsigned long gene = std::strtoul(gene_hex.c_str(), &end, 16);
            if (*end != '\0' || gene > 0xffffffffUL)
                continue;
            const double v = std::strtod(t.c_str(), &end);
            if (*end != '\0')
                continue;
            known_[static_cast<uint32_t>(gene)] = v;
        }
        out_ = std::fopen(path.c_str(), "a");
        if (!out_)
            fail(OFL_EINVAL, "tune cache: cannot open " + path + " for appending");
    }
    ~TuneCache() {
        if (out_)
            std::fclose(out_);
    }
    TuneCache(const TuneCache &) = delete;
    TuneCache &operator=(const TuneCache &) = delete;

    bool lookup(uint32_t gene, double *t) const {
        auto it = known_.find(gene);
        if (it == known_.end())
            return false;
        *t = it->second;
        return true;
    }
    void record(uint32_t gene, double t) {
        known_[gene] = t;
        if (!out_)
            return;
        std::fprintf(out_, "ofl-tune 1 %s %x %.17g\n", key_.c_str(), gene, t);
        std::fflush(out_);
    }

  private:
    std::string key_;
    std::map<uint32_t, double> known_;
    FILE *out_ = nullptr;
};

std::string cache_path() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    return g_cache_path;
}

std::string device_key(int device) {
    std::string arch = device_arch(device) + "/" + std::to_string(device_cu_count(device)) + "cu";
    for (char &c : arch)
        if (c == ' ' || c == '\t')
            c = '_';
    return arch;
}

std::string ga_key(const ofl_ga_params &ga) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "probe%d;rep%d;tol%.6g", ga.probe_iters, ga.repeats, ga.tolerance);
    return buf;
}

std::string grid_key(const ofl_grid *g, const ofl_ga_params &ga) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "grid;%dx%dx%d;fmt%d;sum%d;fuse%u;align%d;", g->I, g->J, g->K, g->fmt, g->sum_mode,
                  g->fusion, g->row_align);
    return buf + ga_key(ga) + ";" + device_key(g->device) + ";" + OFL_SOURCE_HASH;
}

std::string batch_key(const ofl_batch *b, const ofl_ga_params &ga) {
    // the grids' shapes and alignments, in batch order, hashed (FNV-1a, 64 bits)
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](int v) {
        for (int s = 0; s < 32; s += 8) {
            h ^= static_cast<uint64_t>((static_cast<unsigned>(v) >> s) & 0xffu);
            h *= 1099511628211ULL;
        }
    };
    for (const ofl_grid *g : b->grids) {
        mix(g->I);
        mix(g->J);
        mix(g->K);
        mix(g->row_align);
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "batch;n%zu;shapes%016llx;fmt%d;sum%d;fuse%u;", b->grids.size(),
                  static_cast<unsigned long long>(h), b->fmt, b->sum_mode, b->fusion);
    return buf + ga_key(ga) + ";" + device_key(b->device) + ";" + OFL_SOURCE_HASH;
}

template <class Eval>
void run_ga(const ofl_ga_params &ga, bool batch, uint32_t seed_gene, TuneCache &cache, Eval &&evaluate,
            ofl_tune_result *out) {
    int from_cache = 0;
    auto cached_eval = [&](uint32_t gene) -> double {
        double t;
        if (cache.lookup(gene, &t)) {
            ++from_cache;
            return t;
        }
        t = evaluate(gene);
        cache.record(gene, t);
        return t;
    };
    const GaOutcome r = ga_search(ga, gene_bits(batch), seed_gene, cached_eval);
    TileCfg t;
    if (!(r.best_t < kInf) || !decode(r.best, batch, &t))
        fail(OFL_ESTATE, "no gene produced a correct result");
    out->best = to_tile(t);
    out->best_ms = r.best_t;
    out->evaluated = r.evaluated;
    out->rejected = r.rejected;
    out->from_cache = from_cache;
}

ofl_ga_params defaults_or(const ofl_ga_params *ga) {
    if (ga)
        return *ga;
    ofl_ga_params d;
    d.population = 16;
    d.generations = 12;
    d.seed = 2011036020ULL;
    d.crossover = 0.9;
    d.mutation = 0.05;
    d.elite = 1;
    d.probe_iters = 5;
    d.repeats = 3;
    d.tolerance = 1e-5;
    return d;
}

// The measuring side of the offload searches: the initial iterate every run
// starts from (nothing on the device, so each run pays the transfers its gene
// needs), the all-CPU result (the original program) each run is checked
// against, and end-to-end runs timed on the host clock.
struct OffloadBench {
    ofl_grid *g;
    int iters;
    float omega;
    double tol;
    int repeats;
    std::vector<float> p0, p_ref;
    double pmax = 0.0, gosa_ref = 0.0, cpu_ms = 0.0;
    unsigned mask0;
    int mode0;
    int level0[3];

    OffloadBench(ofl_grid *grid, int it, float w, double tolerance, int reps)
        : g(grid), iters(it), omega(w), tol(tolerance), repeats(reps) {
        std::vector<Xfer> xs;
        plan_sync_host(-1, g->valid, xs);
        grid_exec(g, xs);
        grid_sync(g);
        p0.assign(g->p, g->p + g->n);
        mask0 = g->mask;
        mode0 = g->mode;
        std::copy(g->level, g->level + 3, level0);
        const int cpu_level[3] = {OFL_LEVEL_K, OFL_LEVEL_K, OFL_LEVEL_K};
        cpu_ms = run(OFL_MASK_ALL_CPU, cpu_level, OFL_XFER_HOISTED, &gosa_ref);
        p_ref.assign(g->p, g->p + g->n);
        for (float v : p_ref)
            pmax = std::max(pmax, static_cast<double>(std::fabs(v)));
    }

    void restore() {
        grid_sync(g);
        std::memcpy(g->p, p0.data(), p0.size() * sizeof(float));
        g->valid = fresh_validity();
    }

    // Put back the caller's regions (after a failure).
    void restore_regions() {
        g->mask = mask0;
        g->mode = mode0;
        std::copy(level0, level0 + 3, g->level);
    }

    // Median of `repeats` end-to-end runs, each from the initial iterate; the
    // result of the last run stays in p and *gosa. With limit_ms > 0 a run
    // still going after limit_ms throws Timeout.
    double run(unsigned mask, const int level[3], int mode, double *gosa, double limit_ms = 0.0) {
        struct ClearDeadline {
            ofl_grid *g;
            ~ClearDeadline() { g->deadline_ns = 0; }
        } clear{g};
        std::vector<double> ms;
        for (int r = 0; r < repeats; ++r) {
            restore();
            g->mask = mask;
            g->mode = mode;
            std::copy(level, level + 3, g->level);
            const auto t0 = std::chrono::steady_clock::now();
            if (limit_ms > 0.0)
                g->deadline_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(t0.time_since_epoch()).count() +
                                 static_cast<long long>(limit_ms * 1e6);
            grid_run_loop(g, iters, omega, 3);
            std::vector<Xfer> xs;
            plan_sync_host(iters, g->valid, xs);
            grid_exec(g, xs);
            *gosa = grid_fetch_gosa(g);
            const auto t1 = std::chrono::steady_clock::now();
            ms.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        std::sort(ms.begin(), ms.end());
        return ms[ms.size() / 2];
    }

    // Does the last run reproduce the original program's result?
    bool matches(double gosa) const {
        double dmax = 0.0;
        for (size_t t = 0; t < g->n; ++t)
            dmax = std::max(dmax, std::fabs(static_cast<double>(g->p[t]) - p_ref[t]));
        return dmax <= tol * std::max(pmax, 1e-300) && std::fabs(gosa - gosa_ref) <= 10.0 * tol * std::fabs(gosa_ref);
    }
};

}  // namespace

}  // namespace ofl

using namespace ofl;

extern "C" {

int ofl_ga_search(int bits, const ofl_ga_params *ga_in, uint32_t seed_gene, ofl_gene_eval eval, void *ctx,
                  ofl_ga_result *out) {
    return guarded(nullptr, [&] {
        if (bits < 1 || bits > 30 || !eval || !out)
            fail(OFL_EINVAL, "bits must be in 1..30 and eval/out must not be NULL");
        const ofl_ga_params ga = defaults_or(ga_in);
        check_params(ga);
        const GaOutcome r = ga_search(ga, bits, seed_gene, [&](uint32_t g) { return eval(g, ctx); });
        out->best_gene = r.best;
        out->best_time = r.best_t;
        out->evaluated = r.evaluated;
        out->rejected = r.rejected;
    });
}

int ofl_grid_search_offload(ofl_grid *g, const ofl_ga_params *ga_in, int iters, float omega,
                            ofl_offload_result *out) {
    return grid_call(g, [&] {
        if (!g || !out)
            fail(OFL_EINVAL, "NULL argument");
        if (g->broken)
            fail(OFL_EDEVICE, "grid handle unusable after an earlier device error");
        if (iters < 1 || !std::isfinite(omega) || omega == 0.f)
            fail(OFL_EINVAL, "iters must be >= 1 and omega finite and non-zero");
        if (g->in_region || g->batch_refs > 0)
            fail(OFL_ESTATE, "close the data region and leave any batch before searching offload genes");
        const ofl_ga_params ga = defaults_or(ga_in);
        check_params(ga);
        OffloadBench bench(g, iters, omega, ga.tolerance, ga.repeats);
        const int whole[3] = {OFL_LEVEL_K, OFL_LEVEL_K, OFL_LEVEL_K};
        auto evaluate = [&](uint32_t gene) -> double {
            const unsigned mask = gene & 7u;
            const int mode = (gene >> 3) & 1u ? OFL_XFER_HOISTED : OFL_XFER_PER_ITER;
            double gosa = 0.0;
            const double ms = bench.run(mask, whole, mode, &gosa);
            return bench.matches(gosa) ? ms : kInf;
        };
        GaOutcome r;
        try {
            r = ga_search(ga, 4, OFL_MASK_ALL_GPU | 8u, evaluate);
        } catch (...) {
            bench.restore();
            bench.restore_regions();
            throw;
        }
        bench.restore();
        if (!(r.best_t < kInf)) {
            bench.restore_regions();
            fail(OFL_ESTATE, "no offload gene reproduced the all-CPU result");
        }
        g->mask = r.best & 7u;
        g->mode = (r.best >> 3) & 1u ? OFL_XFER_HOISTED : OFL_XFER_PER_ITER;
        std::copy(whole, whole + 3, g->level);
        out->mask = g->mask;
        out->xfer_mode = g->mode;
        out->best_ms = r.best_t;
        out->cpu_ms = bench.cpu_ms;
        out->evaluated = r.evaluated;
        out->rejected = r.rejected;
    });
}

int ofl_grid_search_loops(ofl_grid *g, const ofl_ga_params *ga_in, int iters, float omega, int xfer_mode,
                          double time_limit_ms, ofl_loop_search_result *out) {
    return grid_call(g, [&] {
        if (!g || !out)
            fail(OFL_EINVAL, "NULL argument");
        if (g->broken)
            fail(OFL_EDEVICE, "grid handle unusable after an earlier device error");
        if (iters < 1 || !std::isfinite(omega) || omega == 0.f)
            fail(OFL_EINVAL, "iters must be >= 1 and omega finite and non-zero");
        if (xfer_mode != OFL_XFER_PER_ITER && xfer_mode != OFL_XFER_HOISTED)
            fail(OFL_EINVAL, "unknown xfer_mode");
        if (!(time_limit_ms == time_limit_ms))
            fail(OFL_EINVAL, "time_limit_ms is NaN");
        if (g->in_region || g->batch_refs > 0)
            fail(OFL_ESTATE, "close the data region and leave any batch before searching loop genes");
        const ofl_ga_params ga = defaults_or(ga_in);
        check_params(ga);
        const int bits = loop_gene_bits(g);
        OffloadBench bench(g, iters, omega, ga.tolerance, ga.repeats);
        const double limit_ms = time_limit_ms > 0.0 ? time_limit_ms : 10.0 * bench.cpu_ms;
        // Genes that open the same regions are one program: measure it once.
        std::map<uint32_t, double> measured;
        int wrong = 0, timed_out = 0;
        auto evaluate = [&](uint32_t gene) -> double {
            unsigned mask = 0;
            int level[3];
            decode_loop_gene(g, gene, &mask, level);
            uint32_t key = mask;
            for (int n = 0; n < 3; ++n)
                if ((mask >> n) & 1u)
                    key |= static_cast<uint32_t>(level[n]) << (3 + 2 * n);
            const auto hit = measured.find(key);
            if (hit != measured.end())
                return hit->second;
            double t = kInf;
            try {
                double gosa = 0.0;
                const double ms = bench.run(mask, level, xfer_mode, &gosa, limit_ms);
                if (bench.matches(gosa))
                    t = ms;
                else
                    wrong += 1;
            } catch (const Timeout &) {
                grid_sync(g);
                timed_out += 1;
            }
            measured[key] = t;
            return t;
        };
        // The original gene offloads every nest whole: each nest's k loop.
        uint32_t seed_gene = 0;
        {
            ofl_loop_info t[OFL_NLOOPS];
            ofl_loop_table(g, t);
            int b = 0;
            for (const ofl_loop_info &x : t) {
                if (!x.parallel)
                    continue;
                if (x.level == OFL_LEVEL_K)
                    seed_gene |= 1u << b;
                b += 1;
            }
        }
        GaOutcome r;
        try {
            r = ga_search(ga, bits, seed_gene, evaluate);
        } catch (...) {
            bench.restore();
            bench.restore_regions();
            throw;
        }
        bench.restore();
        if (!(r.best_t < kInf)) {
            bench.restore_regions();
            fail(OFL_ESTATE, "no loop gene reproduced the all-CPU result within the time limit");
        }
        unsigned mask = 0;
        int level[3];
        decode_loop_gene(g, r.best, &mask, level);
        g->mask = mask;
        g->mode = xfer_mode;
        std::copy(level, level + 3, g->level);
        out->gene = r.best;
        out->mask = mask;
        std::copy(level, level + 3, out->level);
        out->gene_bits = bits;
        out->best_ms = r.best_t;
        out->cpu_ms = bench.cpu_ms;
        out->evaluated = r.evaluated;
        out->patterns = static_cast<int>(measured.size());
        out->rejected = wrong;
        out->timed_out = timed_out;
    });
}

int ofl_set_tune_cache(const char *path) {
    return guarded(nullptr, [&] {
        std::string p = path ? path : "";
        if (p.find('\n') != std::string::npos)
            fail(OFL_EINVAL, "tune cache path holds a newline");
        std::lock_guard<std::mutex> lock(g_cache_mu);
        g_cache_path = p;
    });
}

int ofl_grid_tune(ofl_grid *g, const ofl_ga_params *ga_in, ofl_tune_result *out) {
    return grid_call(g, [&] {
        if (!g || !out)
            fail(OFL_EINVAL, "NULL argument");
        if (g->broken)
            fail(OFL_EDEVICE, "grid handle unusable after an earlier device error");
        const ofl_ga_params ga = defaults_or(ga_in);
        check_params(ga);
        // Bring p home and keep a copy: the timing runs iterate on the device.
        grid_ensure_device(g);
        {
            std::vector<Xfer> xs;
            plan_sync_host(-1, g->valid, xs);
            grid_exec(g, xs);
            grid_sync(g);
        }
        std::vector<float> saved(g->p, g->p + g->n);
        const unsigned mask = g->mask;
        const int mode = g->mode;
        const TileCfg old = g->tile;
        g->mask = OFL_MASK_ALL_GPU;
        g->mode = OFL_XFER_HOISTED;
        std::map<uint32_t, bool> checked;
        auto evaluate = [&](uint32_t gene) -> double {
            TileCfg t;
            if (!decode(gene, false, &t))
                return kInf;
            const uint32_t key = gene & 0xfffu;
            auto it = checked.find(key);
            const bool ok = it != checked.end()
                                ? it->second
                                : (checked[key] = tile_correct(t, false, g->fmt, g->sum_mode, g->device, ga.tolerance));
            if (!ok)
                return kInf;
            return time_grid(g, t, ga);
        };
        ofl_tune_result res{};
        try {
            TuneCache cache(cache_path(), grid_key(g, ga));
            run_ga(ga, false, encode(old, false), cache, evaluate, &res);
        } catch (...) {
            g->mask = mask;
            g->mode = mode;
            g->tile = old;
            throw;
        }
        grid_sync(g);
        std::memcpy(g->p, saved.data(), saved.size() * sizeof(float));
        g->valid.host[OFL_ARR_P] = 1;
        g->valid.dev[OFL_ARR_P] = 0;
        g->mask = mask;
        g->mode = mode;
        g->tile = to_cfg(res.best);
        g->tile_chosen = true;
        *out = res;
    });
}

int ofl_batch_tune(ofl_batch *b, const ofl_ga_params *ga_in, ofl_tune_result *out) {
    return batch_call(b, [&] {
        if (!b || !out)
            fail(OFL_EINVAL, "NULL argument");
        const ofl_ga_params ga = defaults_or(ga_in);
        check_params(ga);
        hip_check(hipSetDevice(b->device), "hipSetDevice");
        std::vector<std::vector<float>> saved;
        for (ofl_grid *g : b->grids) {
            std::vector<Xfer> xs;
            plan_sync_host(-1, g->valid, xs);
            grid_exec(g, xs);
            grid_sync(g);
            saved.emplace_back(g->p, g->p + g->n);
        }
        batch_prepare(b);
        const TileCfg old = b->tile;
        std::map<uint32_t, bool> checked;
        auto evaluate = [&](uint32_t gene) -> double {
            TileCfg t;
            if (!decode(gene, true, &t))
                return kInf;
            auto it = checked.find(gene);
            const bool ok = it != checked.end()
                                ? it->second
                                : (checked[gene] = tile_correct(t, true, b->fmt, b->sum_mode, b->device, ga.tolerance));
            if (!ok)
                return kInf;
            const double ms = time_batch(b, t, ga);
            batch_mark_done(b, 0);
            return ms;
        };
        ofl_tune_result res{};
        TuneCache cache(cache_path(), batch_key(b, ga));
        run_ga(ga, true, encode(old, true), cache, evaluate, &res);
        const ofl_tile best = res.best;
        if (ofl_batch_set_tile(b, &best) != OFL_OK)
            fail(OFL_EINVAL, ofl_last_error());
        for (size_t t = 0; t < b->grids.size(); ++t) {
            ofl_grid *g = b->grids[t];
            std::memcpy(g->p, saved[t].data(), saved[t].size() * sizeof(float));
            g->valid.host[OFL_ARR_P] = 1;
            g->valid.dev[OFL_ARR_P] = 0;
            g->valid.dev[OFL_ARR_WRK2] = 1;
            g->valid.host[OFL_ARR_WRK2] = 0;
        }
        *out = res;
    });
}

}  // extern "C"
