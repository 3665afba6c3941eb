// Plans: one parallel-tempering cycle (sweep and measurement, then an exchange pass)
// of several ensembles, captured once into a HIP graph inside the library and replayed
// by hsg_plan_run.  Each ensemble's work is forked onto a capture stream of its own, so
// the size classes of an uneven batch run concurrently in the graph; the whole cycle
// is one graph launch.  Exchanges that alternate between even and odd pairs keep two
// graphs (one per parity) and the plan remembers which parity comes next.  Graphs of
// 2, 4, ... cycles (up to the largest power of two <= `unroll`, default 16) cover
// longer runs with few launches, so the per-launch cost of a graph, and the drain of
// its streams at its end, is paid once per many cycles.
//
// The cycle's settings come from a small JSON object (a flat set of keys whose values
// are numbers, strings or arrays of numbers); unknown keys are refused.
#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hsg_device.h"
#include "hsg_launch.h"

namespace {

// Failures are reported like every other entry point's (hsg_last_error).
hsg_status plan_fail(hsg_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hsg_status plan_fail(hsg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    hsg::set_last_error(buf);
    return code;
}

// ---------------------------------------------------------------- settings
struct Settings {
    int exchange = 0;  // 0 plain, 1 annealed, 2 decimated, 3 cooling / heating, 4 none
    int pairing = -2;  // -2: the exchange's default; -1: alternate odd / even pairs
    int n_hb = 1, n_or = 3;
    int anneal_n_hb = -1, anneal_n_or = -1;
    int measure = 1;
    int streams = 1;
    int split = 1;   // parts of consecutive samples per ensemble, each on a stream of its own
    std::vector<int> stream_of;  // capture stream of each ensemble (default: one each)
    int unroll = 16;  // the longest graph: the largest power of two <= unroll cycles
    double eps = 0.0;
    std::vector<double> eps_pairs;  // per pair of every ensemble, ensembles in order
    std::vector<int> path, block_threads, replicas_per_block, flags;  // one value or one per ensemble
};

struct Parser {
    const char* p;
    std::string err;

    void ws() {
        while (*p && std::isspace(static_cast<unsigned char>(*p))) ++p;
    }
    bool expect(char c) {
        ws();
        if (*p != c) {
            err = std::string("expected '") + c + "'";
            return false;
        }
        ++p;
        return true;
    }
    bool string(std::string& out) {
        ws();
        if (*p != '"') {
            err = "expected a string";
            return false;
        }
        ++p;
        out.clear();
        while (*p && *p != '"') {
            if (*p == '\\') {
                err = "escapes are not supported";
                return false;
            }
            out += *p++;
        }
        if (*p != '"') {
            err = "unterminated string";
            return false;
        }
        ++p;
        return true;
    }
    bool number(double& out) {
        ws();
        char* end = nullptr;
        out = std::strtod(p, &end);
        if (end == p || !std::isfinite(out)) {
            err = "expected a finite number";
            return false;
        }
        p = end;
        return true;
    }
    // a number, or an array of numbers
    bool numbers(std::vector<double>& out) {
        ws();
        out.clear();
        if (*p != '[') {
            double v;
            if (!number(v)) return false;
            out.push_back(v);
            return true;
        }
        ++p;
        ws();
        if (*p == ']') {
            ++p;
            return true;
        }
        for (;;) {
            double v;
            if (!number(v)) return false;
            out.push_back(v);
            ws();
            if (*p == ',') {
                ++p;
                continue;
            }
            return expect(']');
        }
    }
};

bool as_int(const std::vector<double>& v, int& out) {
    if (v.size() != 1 || v[0] != std::floor(v[0]) || std::fabs(v[0]) > 1e9) return false;
    out = static_cast<int>(v[0]);
    return true;
}

bool as_ints(const std::vector<double>& v, std::vector<int>& out) {
    out.clear();
    for (double x : v) {
        if (x != std::floor(x) || std::fabs(x) > 1e9) return false;
        out.push_back(static_cast<int>(x));
    }
    return true;
}

hsg_status parse(const char* json, Settings& s) {
    if (!json || !*json) return HSG_OK;
    Parser ps{json, ""};
    if (!ps.expect('{')) return plan_fail(HSG_ERR_INVALID, "plan settings: %s", ps.err.c_str());
    ps.ws();
    if (*ps.p == '}') {
        ++ps.p;
    } else {
        for (;;) {
            std::string key;
            if (!ps.string(key) || !ps.expect(':'))
                return plan_fail(HSG_ERR_INVALID, "plan settings: %s", ps.err.c_str());
            ps.ws();
            if (key == "exchange") {
                std::string v;
                if (!ps.string(v)) return plan_fail(HSG_ERR_INVALID, "plan settings: exchange: %s", ps.err.c_str());
                if (v == "plain") s.exchange = 0;
                else if (v == "anneal") s.exchange = 1;
                else if (v == "decimate") s.exchange = 2;
                else if (v == "coolheat") s.exchange = 3;
                else if (v == "none") s.exchange = 4;
                else return plan_fail(HSG_ERR_INVALID, "plan settings: unknown exchange \"%s\"", v.c_str());
            } else {
                std::vector<double> v;
                if (!ps.numbers(v)) return plan_fail(HSG_ERR_INVALID, "plan settings: %s: %s", key.c_str(), ps.err.c_str());
                bool ok = true;
                if (key == "pairing") ok = as_int(v, s.pairing);
                else if (key == "n_hb") ok = as_int(v, s.n_hb);
                else if (key == "n_or") ok = as_int(v, s.n_or);
                else if (key == "anneal_n_hb") ok = as_int(v, s.anneal_n_hb);
                else if (key == "anneal_n_or") ok = as_int(v, s.anneal_n_or);
                else if (key == "measure") ok = as_int(v, s.measure);
                else if (key == "streams") ok = as_int(v, s.streams);
                else if (key == "split") ok = as_int(v, s.split);
                else if (key == "stream") ok = as_ints(v, s.stream_of);
                else if (key == "unroll") ok = as_int(v, s.unroll);
                else if (key == "eps") {
                    if (v.size() == 1) s.eps = v[0];
                    else s.eps_pairs = v;
                } else if (key == "path") ok = as_ints(v, s.path);
                else if (key == "block_threads") ok = as_ints(v, s.block_threads);
                else if (key == "replicas_per_block") ok = as_ints(v, s.replicas_per_block);
                else if (key == "flags") ok = as_ints(v, s.flags);
                else return plan_fail(HSG_ERR_INVALID, "plan settings: unknown key \"%s\"", key.c_str());
                if (!ok) return plan_fail(HSG_ERR_INVALID, "plan settings: %s must be an integer", key.c_str());
            }
            ps.ws();
            if (*ps.p == ',') {
                ++ps.p;
                continue;
            }
            if (!ps.expect('}')) return plan_fail(HSG_ERR_INVALID, "plan settings: %s", ps.err.c_str());
            break;
        }
    }
    ps.ws();
    if (*ps.p) return plan_fail(HSG_ERR_INVALID, "plan settings: trailing characters");
    return HSG_OK;
}

// ---------------------------------------------------------------- the plan
struct Plan {
    std::vector<hsg_ensemble> ens;
    Settings set;
    std::vector<hsg_tuning> tune;
    std::vector<bool> tuned;
    std::vector<int> group;  // capture stream of each ensemble of the plan
    std::vector<size_t> eps_off;  // first per-pair eps of each ensemble of the plan
    std::vector<bool> is_part;    // a part of a split ensemble (scratch: the plan's own)
    void* part_scratch = nullptr;  // the parts' scratch (library-owned)
    bool alternating = false;
    int next_parity = 0;
    int device = 0;
    double* eps_dev = nullptr;  // per-pair cooling / heating parameters (library-owned)
    // [2 j + p]: 2^j cycles, the first with exchange parity p (p = 0 only unless the
    // plan alternates), j < n_sizes
    static constexpr int kMaxSizes = 9;
    int n_sizes = 1;
    hipGraphExec_t exec[2 * kMaxSizes] = {};
    hipGraph_t graph[2 * kMaxSizes] = {};
};

// Samples [s0, s0 + h) of ensemble e as an ensemble of their own: the same arrays at
// the samples' offsets (layouts of the header: spins [S][C][R][3][2][N/2], couplings
// [S][3][2][N/2], per-slot arrays [S][C][R], per-chain [S][C], per-pair [S][C][R-1][2],
// Q [S][R][3][3], chi [S][R]) and the stream offsets advanced, so that every random
// number, and with it every result, is the one of the whole ensemble.  Its scratch is
// set by the plan (exchanges keep only intermediate values there within a call).
hsg_ensemble sub_ensemble(const hsg_ensemble& e, int s0, int h) {
    hsg_ensemble p = e;
    const size_t C = static_cast<size_t>(e.n_chains), R = static_cast<size_t>(e.n_temps);
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L, ts = e.precision == HSG_FP64 ? 8 : 4;
    const size_t chain0 = static_cast<size_t>(s0) * C, slot0 = chain0 * R;
    auto at = [](auto* ptr, size_t n) { return ptr ? ptr + n : ptr; };
    p.n_samples = h;
    p.sample_base = e.sample_base + static_cast<uint32_t>(s0);
    p.chain_base = e.chain_base + static_cast<uint32_t>(chain0);
    p.slot_base = e.slot_base + static_cast<uint32_t>(slot0);
    p.spins = e.spins ? static_cast<void*>(static_cast<unsigned char*>(e.spins) + slot0 * 3 * N * ts) : nullptr;
    p.couplings = e.couplings
                      ? static_cast<void*>(static_cast<unsigned char*>(e.couplings) + static_cast<size_t>(s0) * 3 * N * ts)
                      : nullptr;
    p.temp_of_slot = at(e.temp_of_slot, slot0);
    p.slot_of_temp = at(e.slot_of_temp, slot0);
    p.energy = at(e.energy, slot0);
    p.sweep_ctr = at(e.sweep_ctr, slot0);
    p.swap_ctr = at(e.swap_ctr, chain0);
    p.swap_stats = at(e.swap_stats, chain0 * (R - 1) * 2);
    p.rt_state = at(e.rt_state, slot0);
    p.rt_trips = at(e.rt_trips, slot0);
    p.work = at(e.work, chain0 * (R - 1) * 2);
    p.Q = at(e.Q, static_cast<size_t>(s0) * R * 9);
    p.chi = at(e.chi, static_cast<size_t>(s0) * R);
    p.e_temp = at(e.e_temp, slot0);
    p.scratch = nullptr;
    return p;
}

// One cycle of ensemble i on stream st: sweep and measurement, then the exchange.
hsg_status enqueue_cycle(const Plan& pl, int i, int parity, hipStream_t st) {
    const hsg_ensemble* e = &pl.ens[i];
    const Settings& s = pl.set;
    void* vs = static_cast<void*>(st);
    hsg_status r;
    if (s.measure && !pl.tuned[i]) {
        r = hsg_sweep_measure(e, 1, 1, s.n_hb, s.n_or, vs);
    } else {
        r = hsg_sweep_tuned(e, 1, 1, s.n_hb, s.n_or, pl.tuned[i] ? &pl.tune[i] : nullptr, vs);
        if (r == HSG_OK && s.measure) r = hsg_measure(e, 1, vs);
    }
    if (r != HSG_OK) return r;
    const int pairing = s.pairing >= 0 ? s.pairing : parity + 1;
    switch (s.exchange) {
    case 0: return hsg_swap(e, 1, pairing, vs);
    case 1: return hsg_anneal_swap(e, 1, parity, s.anneal_n_hb, s.anneal_n_or, vs);
    case 2: return hsg_decimate_swap(e, 1, pairing, vs);
    case 3:
        if (pl.eps_dev) return hsg_coolheat_swap_pairs(e, 1, pairing, pl.eps_dev + pl.eps_off[i], vs);
        return hsg_coolheat_swap(e, 1, pairing, s.eps, vs);
    default: return HSG_OK;
    }
}

// Capture n_cyc cycles of every ensemble, the first with exchange parity `parity`
// (alternating from there for alternating plans), into pl.graph/exec[slot].
hsg_status capture(Plan& pl, int parity, int n_cyc, int slot) {
    const int n = static_cast<int>(pl.ens.size());
    int n_side = 0;
    if (pl.set.streams != 0)
        for (int g : pl.group) n_side = g + 1 > n_side ? g + 1 : n_side;
    const bool fork = n_side > 1;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side(fork ? n_side : 0, nullptr);
    std::vector<hipEvent_t> join(fork ? n_side : 0, nullptr);
    hipEvent_t start = nullptr;
    hsg_status result = HSG_OK;
    hipError_t err = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    for (int i = 0; err == hipSuccess && i < static_cast<int>(side.size()); ++i) {
        err = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    }
    if (err == hipSuccess && fork) err = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    if (err == hipSuccess) err = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (err != hipSuccess) {
        result = plan_fail(HSG_ERR_DEVICE, "plan capture setup: %s", hipGetErrorString(err));
    } else {
        if (fork) err = hipEventRecord(start, cap);
        for (size_t g = 0; g < side.size() && err == hipSuccess; ++g) err = hipStreamWaitEvent(side[g], start, 0);
        // each ensemble's cycles follow one another on its stream (ensembles that share a
        // stream one after another, in order); the streams join at the end
        for (int i = 0; i < n && err == hipSuccess && result == HSG_OK; ++i) {
            hipStream_t st = fork ? side[pl.group[i]] : cap;
            int par = parity;
            for (int c = 0; c < n_cyc && result == HSG_OK; ++c) {
                result = enqueue_cycle(pl, i, par, st);
                if (pl.alternating) par ^= 1;
            }
            if (result != HSG_OK) {
                const std::string why = hsg_last_error();
                plan_fail(result, "plan capture, ensemble %d: %s", i, why.c_str());
                break;
            }
        }
        for (size_t g = 0; g < side.size() && err == hipSuccess && result == HSG_OK; ++g) {
            err = hipEventRecord(join[g], side[g]);
            if (err == hipSuccess) err = hipStreamWaitEvent(cap, join[g], 0);
        }
        hipGraph_t g = nullptr;
        const hipError_t end = hipStreamEndCapture(cap, &g);
        if (result == HSG_OK && err != hipSuccess)
            result = plan_fail(HSG_ERR_DEVICE, "plan capture: %s", hipGetErrorString(err));
        if (result == HSG_OK && end != hipSuccess)
            result = plan_fail(HSG_ERR_DEVICE, "plan capture end: %s", hipGetErrorString(end));
        if (result == HSG_OK) {
            err = hipGraphInstantiate(&pl.exec[slot], g, nullptr, nullptr, 0);
            if (err != hipSuccess) result = plan_fail(HSG_ERR_DEVICE, "plan instantiate: %s", hipGetErrorString(err));
        }
        if (result == HSG_OK) pl.graph[slot] = g;
        else if (g) (void)hipGraphDestroy(g);
    }
    for (size_t i = 0; i < side.size(); ++i) {
        if (join[i]) (void)hipEventDestroy(join[i]);
        if (side[i]) (void)hipStreamDestroy(side[i]);
    }
    if (start) (void)hipEventDestroy(start);
    if (cap) (void)hipStreamDestroy(cap);
    return result;
}

void release(Plan* pl) {
    if (!pl) return;
    int cur = 0;
    const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != pl->device;
    if (switch_dev) (void)hipSetDevice(pl->device);
    for (int k = 0; k < 2 * Plan::kMaxSizes; ++k) {
        if (pl->exec[k]) (void)hipGraphExecDestroy(pl->exec[k]);
        if (pl->graph[k]) (void)hipGraphDestroy(pl->graph[k]);
    }
    if (pl->eps_dev) (void)hipFree(pl->eps_dev);
    if (pl->part_scratch) (void)hipFree(pl->part_scratch);
    if (switch_dev) (void)hipSetDevice(cur);
    delete pl;
}

}  // namespace

extern "C" {

hsg_status hsg_plan_create(const hsg_ensemble* ens, int n_ens, const char* tuning_json, void** plan) {
    if (!plan) return plan_fail(HSG_ERR_INVALID, "plan: the output pointer is NULL");
    *plan = nullptr;
    if (!ens || n_ens < 1 || n_ens > 64) return plan_fail(HSG_ERR_INVALID, "plan: need 1 to 64 ensembles");
    Plan* pl = new Plan();
    Settings& s = pl->set;
    hsg_status r = parse(tuning_json, s);
    if (r != HSG_OK) {
        delete pl;
        return r;
    }
    if (s.anneal_n_hb < 0) s.anneal_n_hb = s.n_hb;
    if (s.anneal_n_or < 0) s.anneal_n_or = s.n_or;
    if (s.pairing == -2) s.pairing = (s.exchange == 0) ? 0 : -1;
    auto bad = [&](const char* msg) {
        delete pl;
        return plan_fail(HSG_ERR_INVALID, "plan settings: %s", msg);
    };
    if (s.pairing < -1 || s.pairing > 2) return bad("pairing must be -1 (alternate), 0, 1 or 2");
    if (s.unroll < 1 || s.unroll > 256) return bad("unroll must be in [1, 256]");
    if (s.split < 1 || s.split > 16) return bad("split must be in [1, 16]");
    if (s.exchange == 1 && s.pairing >= 0) return bad("the annealed exchange alternates even and odd pairs (pairing -1)");
    if (s.n_hb < 0 || s.n_hb > 127 || s.n_or < 0 || s.n_hb + s.n_or < 1) return bad("need 0 <= n_hb <= 127, n_or >= 0, n_hb + n_or >= 1");
    if (!(s.eps >= 0.0)) return bad("eps must be >= 0");
    pl->ens.assign(ens, ens + n_ens);
    pl->alternating = s.exchange != 4 && s.pairing < 0;
    size_t n_pairs = 0;
    for (int i = 0; i < n_ens; ++i) n_pairs += static_cast<size_t>(ens[i].n_temps > 0 ? ens[i].n_temps - 1 : 0);
    if (!s.eps_pairs.empty()) {
        if (s.exchange != 3) return bad("per-pair eps is for the cooling / heating exchange");
        if (s.eps_pairs.size() != n_pairs) return bad("eps needs one value per pair of every ensemble, in order");
        for (double v : s.eps_pairs)
            if (!(v >= 0.0)) return bad("eps must be >= 0");
    }
    auto per_ens = [&](const std::vector<int>& v, int i) { return v.empty() ? 0 : (v.size() == 1 ? v[0] : v[i]); };
    for (const auto* v : {&s.path, &s.block_threads, &s.replicas_per_block, &s.flags})
        if (v->size() > 1 && static_cast<int>(v->size()) != n_ens) return bad("tuning arrays need one value per ensemble");
    pl->tune.resize(n_ens);
    pl->tuned.resize(n_ens);
    for (int i = 0; i < n_ens; ++i) {
        hsg_tuning t{per_ens(s.path, i), per_ens(s.block_threads, i), per_ens(s.replicas_per_block, i),
                     per_ens(s.flags, i)};
        pl->tune[i] = t;
        pl->tuned[i] = t.path != 0 || t.block_threads != 0 || t.replicas_per_block != 0 || t.flags != 0;
    }
    if (s.split > 1) {
        // each ensemble of at least two samples as `split` parts of consecutive samples
        // (as equal as the count allows), each captured on a stream of its own: a
        // part's exchange and the start and end of its launches overlap the other
        // parts' sweeps.  Allowed for the LDS-resident sweeps (L <= 16), which, like the
        // plain exchange, use no scratch.
        std::vector<hsg_ensemble> parts;
        std::vector<hsg_tuning> ptune;
        std::vector<bool> ptuned, part;
        std::vector<size_t> poff;
        size_t off = 0;
        for (int i = 0; i < n_ens; ++i) {
            const hsg_ensemble& e = ens[i];
            const int path = pl->tune[i].path;
            if (e.L > 16 || (path != 0 && path != 3 && path != 6)) return bad("split needs LDS-resident sweeps (L <= 16; path 0, 3 or 6)");
            const int k = e.n_samples < s.split ? (e.n_samples > 0 ? e.n_samples : 1) : s.split;
            for (int q = 0; q < k; ++q) {
                const int s0 = static_cast<int>(static_cast<long long>(e.n_samples) * q / k);
                const int s1 = static_cast<int>(static_cast<long long>(e.n_samples) * (q + 1) / k);
                parts.push_back(k > 1 ? sub_ensemble(e, s0, s1 - s0) : e);
                ptune.push_back(pl->tune[i]);
                ptuned.push_back(pl->tuned[i]);
                part.push_back(k > 1);
                poff.push_back(off);
            }
            off += static_cast<size_t>(e.n_temps > 0 ? e.n_temps - 1 : 0);
        }
        pl->ens = parts;
        pl->tune = ptune;
        pl->tuned = ptuned;
        pl->is_part = part;
        pl->eps_off = poff;
    } else {
        size_t off = 0;
        for (int i = 0; i < n_ens; ++i) {
            pl->eps_off.push_back(off);
            pl->is_part.push_back(false);
            off += static_cast<size_t>(ens[i].n_temps > 0 ? ens[i].n_temps - 1 : 0);
        }
    }
    // capture streams: one per ensemble (and per part of a split ensemble), or the
    // caller's grouping ("stream": one index per ensemble; ensembles of one group run one
    // after another on one stream, the groups side by side)
    if (!s.stream_of.empty()) {
        if (s.split > 1) return bad("stream and split do not combine");
        if (static_cast<int>(s.stream_of.size()) != n_ens) return bad("stream needs one index per ensemble");
        for (int g : s.stream_of)
            if (g < 0 || g >= n_ens) return bad("stream indices must be in [0, number of ensembles)");
        pl->group = s.stream_of;
    } else {
        pl->group.resize(pl->ens.size());
        for (size_t i = 0; i < pl->ens.size(); ++i) pl->group[i] = static_cast<int>(i);
    }
    hipError_t err = hipGetDevice(&pl->device);
    if (err != hipSuccess) {
        delete pl;
        return plan_fail(HSG_ERR_DEVICE, "plan: %s", hipGetErrorString(err));
    }
    if (!s.eps_pairs.empty()) {
        err = hipMalloc(&pl->eps_dev, s.eps_pairs.size() * sizeof(double));
        if (err == hipSuccess)
            err = hipMemcpy(pl->eps_dev, s.eps_pairs.data(), s.eps_pairs.size() * sizeof(double),
                            hipMemcpyHostToDevice);
        if (err != hipSuccess) {
            release(pl);
            return plan_fail(HSG_ERR_DEVICE, "plan: per-pair eps: %s", hipGetErrorString(err));
        }
    }
    // the parts of split ensembles get scratch of their own (one library-owned buffer,
    // cleared once) where the exchange uses scratch: the annealed exchange's candidates,
    // the decimated exchange's partial sums, the cooling / heating exchange's candidates
    // and flags, all of them intermediate values within one call
    if (s.split > 1 && (s.exchange == 1 || s.exchange == 2 || s.exchange == 3)) {
        size_t total = 0;
        std::vector<size_t> at(pl->ens.size(), 0);
        for (size_t i = 0; i < pl->ens.size(); ++i) {
            if (!pl->is_part[i]) continue;
            at[i] = total;
            total += (hsg_scratch_bytes(&pl->ens[i]) + 255) & ~static_cast<size_t>(255);
        }
        if (total > 0) {
            hipStream_t z = nullptr;
            err = hipMalloc(&pl->part_scratch, total);
            if (err == hipSuccess) err = hipStreamCreateWithFlags(&z, hipStreamNonBlocking);
            if (err == hipSuccess) err = hipMemsetAsync(pl->part_scratch, 0, total, z);
            if (err == hipSuccess) err = hipStreamSynchronize(z);
            if (z) (void)hipStreamDestroy(z);
            if (err != hipSuccess) {
                release(pl);
                return plan_fail(HSG_ERR_DEVICE, "plan: scratch of the split parts: %s", hipGetErrorString(err));
            }
            for (size_t i = 0; i < pl->ens.size(); ++i)
                if (pl->is_part[i]) pl->ens[i].scratch = static_cast<unsigned char*>(pl->part_scratch) + at[i];
        }
    }
    // graphs of 1, 2, 4, ... cycles up to the largest power of two <= unroll, so that a
    // run of n cycles is at most log2 graph launches (each launch drains the streams
    // before the next can start); alternating plans keep one per starting parity
    while (pl->n_sizes < Plan::kMaxSizes && (2 << (pl->n_sizes - 1)) <= s.unroll) ++pl->n_sizes;
    for (int j = 0; j < pl->n_sizes && r == HSG_OK; ++j) {
        r = capture(*pl, 0, 1 << j, 2 * j);
        if (r == HSG_OK && pl->alternating) r = capture(*pl, 1, 1 << j, 2 * j + 1);
    }
    if (r != HSG_OK) {
        release(pl);
        return r;
    }
    *plan = pl;
    hsg::set_last_error("");
    return HSG_OK;
}

hsg_status hsg_plan_run(void* plan, int n_cycles, void* stream) {
    if (!plan) return plan_fail(HSG_ERR_INVALID, "plan: NULL plan");
    if (n_cycles < 0) return plan_fail(HSG_ERR_INVALID, "plan: n_cycles must be >= 0");
    Plan* pl = static_cast<Plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int left = n_cycles;
    while (left > 0) {
        int j = pl->n_sizes - 1;  // the longest graph that fits what is left
        while ((1 << j) > left) --j;
        const int g = 2 * j + (pl->alternating ? pl->next_parity : 0);
        const hipError_t err = hipGraphLaunch(pl->exec[g], st);
        if (err != hipSuccess) return plan_fail(HSG_ERR_DEVICE, "plan run: %s", hipGetErrorString(err));
        if (pl->alternating) pl->next_parity ^= ((1 << j) & 1);
        left -= 1 << j;
    }
    hsg::set_last_error("");
    return HSG_OK;
}

int hsg_plan_next_parity(const void* plan) {
    return plan ? static_cast<const Plan*>(plan)->next_parity : -1;
}

hsg_status hsg_plan_set_next_parity(void* plan, int parity) {
    if (!plan || parity < 0 || parity > 1) return plan_fail(HSG_ERR_INVALID, "plan: bad plan or parity");
    static_cast<Plan*>(plan)->next_parity = parity;
    return HSG_OK;
}

hsg_status hsg_plan_destroy(void* plan) {
    release(static_cast<Plan*>(plan));
    return HSG_OK;
}

}  // extern "C"
