// Tuning table of the bound kernels' runtime parameters (argmin tile, data
// split, waves per workgroup, the l2 filter and query order flags): lookup, lip_tune_get / lip_tune_set and
// the JSON cache (lip_tune_save / lip_tune_load, LIPFIT_TUNE_CACHE).
//
// Key: (d, number of monotone coordinates, norm, size class of n, size class
// of q).  A size class is floor(log2(v)) / 2, so the sizes of one class are
// within a factor of 4 of each other; class -1 in both positions is an entry
// set for every size, consulted when the exact class has none.  lip_autotune
// stores its result under the class of the sizes it timed.
//
// Cache file (one JSON object):
//   {"format": "lipfit-tune-1", "entries": [
//     {"arch": "gfx950", "d": 4, "n_mon": 2, "norm": 2, "n_class": 8,
//      "q_class": 9, "tile": 32, "split": 8, "waves": 4, "flags": 1}, ...]}
// Entries of another architecture are kept in the file but not loaded.
#include <ctype.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "host_common.hpp"

namespace lip {

namespace {

typedef std::tuple<int, int, int, int, int> TuneKey;

std::mutex g_mu;
std::map<TuneKey, lip_tile_cfg> g_table;
bool g_env_loaded = false;

int size_class(int64_t v)
{
    if (v <= 0) return -1;
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= v) ++b;
    return b / 2;
}

bool cfg_valid(const lip_tile_cfg &c)
{
    return c.tile >= 8 && c.tile <= kMaxTile && c.tile % 8 == 0 && c.split >= 1 &&
           c.split <= kMaxChunks && c.waves >= 1 && c.waves <= kMaxFwdWaves &&
           (c.flags & ~(LIP_TILE_L2_FILTER | LIP_TILE_QUERY_ORDER)) == 0;
}

// Architecture name of the current device without feature suffixes
// ("gfx950"), or "" when there is none.
std::string current_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return std::string();
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// ---- a reader for the cache's own small JSON form ----------------------------

struct Reader {
    const char *p, *end;
    void ws()
    {
        while (p < end && isspace((unsigned char)*p)) ++p;
    }
    bool lit(char c)
    {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string *out)
    {
        ws();
        if (p >= end || *p != '"') return false;
        ++p;
        std::string s;
        while (p < end && *p != '"') {
            if (*p == '\\') return false;  // the cache never escapes
            s.push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        *out = s;
        return true;
    }
    bool num(long long *out)
    {
        ws();
        const char *b = p;
        if (p < end && (*p == '-' || *p == '+')) ++p;
        while (p < end && isdigit((unsigned char)*p)) ++p;
        if (p == b) return false;
        *out = strtoll(std::string(b, p).c_str(), nullptr, 10);
        return true;
    }
};

struct Entry {
    std::string arch;
    long long d = -1, n_mon = -1, norm = -1, n_class = -2, q_class = -2, tile = -1, split = -1,
              waves = -1, flags = 0;
};

bool read_entry(Reader &r, Entry *e)
{
    if (!r.lit('{')) return false;
    if (r.lit('}')) return true;
    for (;;) {
        std::string key;
        if (!r.str(&key) || !r.lit(':')) return false;
        if (key == "arch") {
            if (!r.str(&e->arch)) return false;
        } else {
            long long v = 0;
            if (!r.num(&v)) return false;
            if (key == "d") e->d = v;
            else if (key == "n_mon") e->n_mon = v;
            else if (key == "norm") e->norm = v;
            else if (key == "n_class") e->n_class = v;
            else if (key == "q_class") e->q_class = v;
            else if (key == "tile") e->tile = v;
            else if (key == "split") e->split = v;
            else if (key == "waves") e->waves = v;
            else if (key == "flags") e->flags = v;
            else return false;
        }
        if (r.lit('}')) return true;
        if (!r.lit(',')) return false;
    }
}

// Parses the whole file first; the table changes only if it all parses.
lip_status load_locked(const char *path, const std::string &arch)
{
    FILE *f = fopen(path, "rb");
    if (!f) return LIP_E_ARG;
    std::string buf;
    char tmp[4096];
    size_t got;
    while ((got = fread(tmp, 1, sizeof tmp, f)) > 0) buf.append(tmp, got);
    fclose(f);
    Reader r{buf.data(), buf.data() + buf.size()};
    std::string key, fmt;
    if (!r.lit('{') || !r.str(&key) || key != "format" || !r.lit(':') || !r.str(&fmt) ||
        fmt != "lipfit-tune-1" || !r.lit(',') || !r.str(&key) || key != "entries" ||
        !r.lit(':') || !r.lit('['))
        return LIP_E_VALUE;
    std::map<TuneKey, lip_tile_cfg> add;
    if (!r.lit(']')) {
        for (;;) {
            Entry e;
            if (!read_entry(r, &e)) return LIP_E_VALUE;
            lip_tile_cfg c{(int32_t)e.tile, (int32_t)e.split, (int32_t)e.waves, (int32_t)e.flags};
            const bool shape_ok = e.d >= 1 && e.d <= kMaxDim && e.n_mon >= 0 && e.n_mon <= e.d &&
                                  e.norm >= LIP_L1 && e.norm <= LIP_LINF && e.n_class >= -1 &&
                                  e.q_class >= -1 && (e.n_class == -1) == (e.q_class == -1);
            if (!shape_ok || !cfg_valid(c)) return LIP_E_VALUE;
            if (e.arch == arch)
                add[TuneKey((int)e.d, (int)e.n_mon, (int)e.norm, (int)e.n_class,
                            (int)e.q_class)] = c;
            if (r.lit(']')) break;
            if (!r.lit(',')) return LIP_E_VALUE;
        }
    }
    if (!r.lit('}')) return LIP_E_VALUE;
    for (auto &kv : add) g_table[kv.first] = kv.second;
    return LIP_OK;
}

lip_status save_locked(const char *path, const std::string &arch)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return LIP_E_ARG;
    fprintf(f, "{\"format\": \"lipfit-tune-1\", \"entries\": [");
    bool first = true;
    for (auto &kv : g_table) {
        const TuneKey &k = kv.first;
        const lip_tile_cfg &c = kv.second;
        fprintf(f,
                "%s\n  {\"arch\": \"%s\", \"d\": %d, \"n_mon\": %d, \"norm\": %d, "
                "\"n_class\": %d, \"q_class\": %d, \"tile\": %d, \"split\": %d, \"waves\": %d, "
                "\"flags\": %d}",
                first ? "" : ",", arch.c_str(), std::get<0>(k), std::get<1>(k), std::get<2>(k),
                std::get<3>(k), std::get<4>(k), c.tile, c.split, c.waves, c.flags);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return LIP_E_ARG;
    }
    return LIP_OK;
}

void env_load_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *path = getenv("LIPFIT_TUNE_CACHE");
    if (path && *path) (void)load_locked(path, current_arch());  // a missing file is no error
}

}  // namespace

lip_tile_cfg tune_lookup(int d, int dm, int norm, int64_t n, int64_t q)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        auto it = g_table.find(TuneKey(d, dm, norm, size_class(n), size_class(q)));
        if (it == g_table.end()) it = g_table.find(TuneKey(d, dm, norm, -1, -1));
        if (it != g_table.end()) return it->second;
    }
    return default_tile_cfg(d, dm, norm, n, q);
}

void tune_autosave()
{
    const char *path = getenv("LIPFIT_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)save_locked(path, current_arch());
}

}  // namespace lip

using namespace lip;

extern "C" {

lip_status lip_tune_get(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                        lip_tile_cfg *cfg)
{
    if (!cfg) return LIP_E_ARG;
    if (d < 1 || d > kMaxDim || n_mon < 0 || n_mon > d) return LIP_E_SHAPE;
    if (norm != LIP_L1 && norm != LIP_L2 && norm != LIP_LINF) return LIP_E_ARG;
    *cfg = tune_lookup(d, n_mon, norm, n, q);
    return LIP_OK;
}

lip_status lip_tune_set(int32_t d, int32_t n_mon, int32_t norm, int64_t n, int64_t q,
                        const lip_tile_cfg *cfg)
{
    if (d < 1 || d > kMaxDim || n_mon < 0 || n_mon > d) return LIP_E_SHAPE;
    if (norm != LIP_L1 && norm != LIP_L2 && norm != LIP_LINF) return LIP_E_ARG;
    if (n < 0 || q < 0 || ((n == 0) != (q == 0))) return LIP_E_SHAPE;
    const TuneKey key(d, n_mon, norm, size_class(n), size_class(q));
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    if (!cfg) {
        g_table.erase(key);
        return LIP_OK;
    }
    if (!cfg_valid(*cfg)) return LIP_E_VALUE;
    g_table[key] = *cfg;
    return LIP_OK;
}

lip_status lip_tune_save(const char *path, const char *arch)
{
    if (!path) return LIP_E_ARG;
    const std::string a = arch ? std::string(arch) : current_arch();
    if (a.empty()) return LIP_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    return save_locked(path, a);
}

lip_status lip_tune_load(const char *path, const char *arch)
{
    if (!path) return LIP_E_ARG;
    const std::string a = arch ? std::string(arch) : current_arch();
    if (a.empty()) return LIP_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    return load_locked(path, a);
}

lip_status lip_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    return LIP_OK;
}

}  // extern "C"
