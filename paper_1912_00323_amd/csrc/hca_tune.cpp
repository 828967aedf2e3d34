// The batch autotuner's persisted choices: one JSON object of entries, each
// the knobs that ran a group of data sets fastest and its time, kept in a
// file (HCA_TUNE_CACHE, else $HOME/.cache/hca_tune.json) that every process
// of the library reads once and rewrites whole after each new entry.
#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "hca_internal.h"

namespace {

struct Entry {
    hca::Tune t;
    double ms = 0;
};

std::mutex g_mu;
bool g_loaded = false;
std::map<std::string, Entry> g_map;

std::string cache_path()
{
    if (const char *e = std::getenv("HCA_TUNE_CACHE")) return e;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/hca_tune.json";
    return "";
}

// Integer (or number) after "name": in an entry's text; false if absent.
bool field(const std::string &obj, const char *name, double *v)
{
    const std::string key = std::string("\"") + name + "\":";
    const size_t at = obj.find(key);
    if (at == std::string::npos) return false;
    *v = std::strtod(obj.c_str() + at + key.size(), nullptr);
    return true;
}

// The file holds {"entries": {"<key>": {"reps": 1, ...}, ...}}, as written
// below; anything else is ignored.
void load_locked()
{
    g_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    std::fclose(f);
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return;
    pos = text.find('{', pos);
    while (pos != std::string::npos) {
        const size_t q0 = text.find('"', pos + 1);
        if (q0 == std::string::npos) break;
        const size_t q1 = text.find('"', q0 + 1);
        const size_t b0 = text.find('{', q1);
        const size_t b1 = text.find('}', b0);
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        const std::string key = text.substr(q0 + 1, q1 - q0 - 1), obj = text.substr(b0, b1 - b0 + 1);
        Entry e;
        double v;
        if (field(obj, "reps", &v)) e.t.reps = (int)v;
        if (field(obj, "lanes", &v)) e.t.lanes = (int)v;
        if (field(obj, "prefix", &v)) e.t.prefix = (int)v;
        if (field(obj, "lists", &v)) e.t.lists = (int)v;
        if (field(obj, "merge_split", &v)) e.t.merge_split = (int)v;
        if (field(obj, "wave_blocks", &v)) e.t.wave_blocks = (int)v;
        if (field(obj, "hash_load", &v)) e.t.hash_load = (int)v;
        if (field(obj, "digit_cap", &v)) e.t.digit_cap = (int)v;
        if (field(obj, "sort_items", &v)) e.t.sort_items = (int)v;
        if (field(obj, "ms", &v)) e.ms = v;
        g_map[key] = e;
        pos = b1 + 1;
        if (text.find('"', pos) == std::string::npos) break;
    }
}

void save_locked()
{
    const std::string path = cache_path();
    if (path.empty()) return;
    // the parent directory (one level, as for $HOME/.cache)
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)::mkdir(path.substr(0, slash).c_str(), 0755);
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\"entries\": {");
    bool first = true;
    for (const auto &kv : g_map) {
        std::string obj = hca::tune_text(kv.second.t);
        obj.pop_back();                       // the closing brace: the time goes in too
        std::fprintf(f, "%s\n  \"%s\": %s, \"ms\": %.6f}", first ? "" : ",", kv.first.c_str(), obj.c_str(),
                     kv.second.ms);
        first = false;
    }
    std::fprintf(f, "\n}}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

namespace hca {

std::string tune_text(const Tune &t)
{
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"reps\": %d, \"lanes\": %d, \"prefix\": %d, \"lists\": %d, \"merge_split\": %d, "
                  "\"wave_blocks\": %d, \"hash_load\": %d, \"digit_cap\": %d, \"sort_items\": %d}",
                  t.reps, t.lanes, t.prefix, t.lists, t.merge_split, t.wave_blocks, t.hash_load, t.digit_cap,
                  t.sort_items);
    return buf;
}

bool tune_cache_get(const std::string &key, Tune *t, double *ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    const auto it = g_map.find(key);
    if (it == g_map.end()) return false;
    *t = it->second.t;
    if (ms) *ms = it->second.ms;
    return true;
}

void tune_cache_put(const std::string &key, const Tune &t, double ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    g_map[key] = Entry{t, ms};
    save_locked();
}

}  // namespace hca
