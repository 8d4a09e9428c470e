// Autotuner cache: a JSON-lines table (one object per grid class) in the file
// the environment variable GS_TUNE_CACHE names. gs_tune and gs_batch_tune
// record their choice; gs_init and gs_batch_init use a recorded choice when
// the caller leaves the launch configuration to the library. The cache is
// advisory: a missing, unreadable or stale entry only means the library's
// defaults are used, and a failed write leaves the tuned handle as it is.
#include "gs_internal.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace gsapi {
namespace {

std::mutex g_cache_mutex;

const char *kind_name(int kind) { return kind == TUNE_BATCH ? "batch" : "single"; }

std::string format_line(const TuneKey &k, const TuneVal &v)
{
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"kind\":\"%s\",\"storage\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"noise\":%d,"
                  "\"tile\":%d,\"tblock\":%d,\"zchunk\":%d,\"ms_per_step\":%.6g}",
                  kind_name(k.kind), k.storage, k.nx, k.ny, k.nz, k.noisy, v.tile, v.tblock, v.zchunk, v.ms_per_step);
    return buf;
}

// Parses one line written by format_line; false for anything else.
bool parse_line(const char *line, TuneKey *k, TuneVal *v)
{
    char kind[16] = {0};
    int n = std::sscanf(line,
                        "{\"kind\":\"%15[a-z]\",\"storage\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"noise\":%d,"
                        "\"tile\":%d,\"tblock\":%d,\"zchunk\":%d,\"ms_per_step\":%lf}",
                        kind, &k->storage, &k->nx, &k->ny, &k->nz, &k->noisy, &v->tile, &v->tblock, &v->zchunk,
                        &v->ms_per_step);
    if (n != 10) return false;
    if (std::strcmp(kind, "single") == 0)
        k->kind = TUNE_SINGLE;
    else if (std::strcmp(kind, "batch") == 0)
        k->kind = TUNE_BATCH;
    else
        return false;
    return true;
}

bool same_key(const TuneKey &a, const TuneKey &b)
{
    return a.kind == b.kind && a.storage == b.storage && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
           a.noisy == b.noisy;
}

std::vector<std::string> read_lines(const char *path)
{
    std::vector<std::string> out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    char buf[512];
    while (std::fgets(buf, sizeof buf, f)) {
        size_t n = std::strlen(buf);
        while (n && (buf[n - 1] == '\n' || buf[n - 1] == '\r')) buf[--n] = 0;
        if (n) out.emplace_back(buf);
    }
    std::fclose(f);
    return out;
}

} // namespace

const char *tune_cache_path()
{
    const char *p = std::getenv("GS_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

bool tune_cache_lookup(const TuneKey &key, TuneVal *val)
{
    const char *path = tune_cache_path();
    if (!path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    bool found = false;
    for (const std::string &l : read_lines(path)) {
        TuneKey k;
        TuneVal v;
        if (parse_line(l.c_str(), &k, &v) && same_key(k, key)) {
            *val = v; // the last entry for a key wins
            found = true;
        }
    }
    return found;
}

bool tune_cache_store(const TuneKey &key, const TuneVal &val)
{
    const char *path = tune_cache_path();
    if (!path) return true;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    std::vector<std::string> keep;
    for (const std::string &l : read_lines(path)) {
        TuneKey k;
        TuneVal v;
        if (parse_line(l.c_str(), &k, &v) && same_key(k, key)) continue;
        keep.push_back(l);
    }
    keep.push_back(format_line(key, val));
    // write a sibling file, then rename it over the table
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (const std::string &l : keep) ok = ok && std::fprintf(f, "%s\n", l.c_str()) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

} // namespace gsapi
