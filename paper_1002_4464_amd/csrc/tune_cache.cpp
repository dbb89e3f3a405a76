// Persisted autotuner results (host code only, no HIP calls).  A text file of one line per key:
//   v1 <device> <key type> <values> <segment class> <classes> {<upper> <L> <s>} x 4
// where the segment class is ceil(log2(max_segment)) of the tuned batch.  Lines are replaced in
// place when a key is stored again; unknown or malformed lines are kept as they are.
#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <string>
#include <vector>

#include "dsort_internal.h"

namespace dsort {

namespace {

std::string key_prefix(const TuneKey &k) {
    char buf[64];
    snprintf(buf, sizeof(buf), " %d %d %u ", k.key_type, k.values ? 1 : 0, k.seg_class);
    std::string dev = k.device;
    for (char &c : dev)
        if (c == ' ' || c == '\n' || c == '\t') c = '_';
    return "v1 " + dev + buf;
}

bool read_lines(const char *path, std::vector<std::string> &lines) {
    FILE *f = fopen(path, "r");
    if (!f) return errno == ENOENT;  // no file yet: empty cache
    char buf[1024];
    while (fgets(buf, sizeof(buf), f)) {
        std::string s(buf);
        while (!s.empty() && (s.back() == '\n' || s.back() == '\r')) s.pop_back();
        if (!s.empty()) lines.push_back(s);
    }
    const bool ok = !ferror(f);
    fclose(f);
    return ok;
}

}  // namespace

uint32_t tune_seg_class(uint64_t max_segment) {
    uint32_t c = 0;
    while (c < 63 && (1ull << c) < max_segment) ++c;
    return c;
}

bool tune_cache_lookup(const char *path, const TuneKey &key, SegTuning &out) {
    std::vector<std::string> lines;
    if (!path || !read_lines(path, lines)) return false;
    const std::string pre = key_prefix(key);
    for (auto it = lines.rbegin(); it != lines.rend(); ++it) {
        if (it->compare(0, pre.size(), pre) != 0) continue;
        SegTuning t;
        unsigned cls = 0;
        unsigned long long up[kMaxSegClasses];
        unsigned L[kMaxSegClasses], s[kMaxSegClasses];
        const int got = sscanf(it->c_str() + pre.size(), "%u %llu %u %u %llu %u %u %llu %u %u %llu %u %u",
                               &cls, &up[0], &L[0], &s[0], &up[1], &L[1], &s[1], &up[2], &L[2],
                               &s[2], &up[3], &L[3], &s[3]);
        if (got != 13 || cls > (unsigned)kMaxSegClasses) return false;
        t.classes = cls;
        for (int q = 0; q < kMaxSegClasses; ++q) {
            t.upper[q] = up[q];
            t.L[q] = L[q];
            t.s[q] = s[q];
        }
        out = t;
        return true;
    }
    return false;
}

bool tune_cache_store(const char *path, const TuneKey &key, const SegTuning &t) {
    if (!path || !*path) return false;
    std::vector<std::string> lines;
    if (!read_lines(path, lines)) return false;
    const std::string pre = key_prefix(key);
    char buf[256];
    snprintf(buf, sizeof(buf), "%u %llu %u %u %llu %u %u %llu %u %u %llu %u %u", t.classes,
             (unsigned long long)t.upper[0], t.L[0], t.s[0], (unsigned long long)t.upper[1],
             t.L[1], t.s[1], (unsigned long long)t.upper[2], t.L[2], t.s[2],
             (unsigned long long)t.upper[3], t.L[3], t.s[3]);
    const std::string line = pre + buf;
    bool replaced = false;
    for (auto &l : lines)
        if (l.compare(0, pre.size(), pre) == 0) {
            l = line;
            replaced = true;
        }
    if (!replaced) lines.push_back(line);
    // write a sibling file and rename it over the cache, so readers never see half a file
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (const auto &l : lines) ok = ok && fprintf(f, "%s\n", l.c_str()) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace dsort
