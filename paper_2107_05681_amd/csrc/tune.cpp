// Autotuner cache and decision rule (host code).
#include "tune.h"

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

namespace meld {

namespace {

// 2: entries carry the sorts' low-phase path (xch); files of version 1 are
// ignored (their decisions predate that choice).
constexpr int kTuneFileVersion = 2;

std::string entry_key(const std::string &op, const std::string &key) { return op + "|" + key; }

std::string to_json(const TuneEntry &e) {
    char buf[512];
    snprintf(buf, sizeof buf,
             "{\"op\": \"%s\", \"key\": \"%s\", \"lo\": %d, \"hi\": %d, \"log_t\": %d, "
             "\"xch\": %d, \"form\": %d, \"ms\": %.6f, \"mixed_lo\": %.6f, \"mixed_hi\": %.6f, "
             "\"trials\": %d}",
             e.op.c_str(), e.key.c_str(), e.lo, e.hi, e.log_t, e.xch, e.form, e.ms, e.mixed_lo,
             e.mixed_hi, e.trials);
    return buf;
}

}  // namespace

bool Tuner::attach(const std::string &path) {
    path_ = path;
    std::ifstream in(path);
    if (!in) return true;  // no file yet: decisions will be written there
    std::string line;
    bool header_ok = false;
    std::map<std::string, TuneEntry> loaded;
    while (std::getline(in, line)) {
        if (line.find("\"version\"") != std::string::npos) {
            int version = 0, runtime = 0;
            char arch[128] = {0};
            if (sscanf(line.c_str(), " {\"version\": %d, \"arch\": \"%127[^\"]\", \"runtime\": %d",
                       &version, arch, &runtime) != 3)
                return false;
            header_ok = version == kTuneFileVersion && arch_ == arch && runtime_ == runtime;
            continue;
        }
        if (line.find("{\"op\"") == std::string::npos) continue;
        char op[32] = {0}, key[128] = {0};
        TuneEntry e;
        if (sscanf(line.c_str(),
                   " {\"op\": \"%31[^\"]\", \"key\": \"%127[^\"]\", \"lo\": %d, \"hi\": %d, "
                   "\"log_t\": %d, \"xch\": %d, \"form\": %d, \"ms\": %lf, \"mixed_lo\": %lf, "
                   "\"mixed_hi\": %lf, \"trials\": %d",
                   op, key, &e.lo, &e.hi, &e.log_t, &e.xch, &e.form, &e.ms, &e.mixed_lo,
                   &e.mixed_hi, &e.trials) != 11)
            return false;
        e.op = op;
        e.key = key;
        loaded[entry_key(e.op, e.key)] = e;
    }
    if (header_ok)
        for (auto &kv : loaded) entries_[kv.first] = kv.second;
    return true;
}

const TuneEntry *Tuner::find(const std::string &op, const std::string &key) const {
    auto it = entries_.find(entry_key(op, key));
    return it == entries_.end() ? nullptr : &it->second;
}

void Tuner::put(const TuneEntry &e) {
    entries_[entry_key(e.op, e.key)] = e;
    if (!path_.empty()) (void)save();
}

std::string Tuner::describe() const {
    std::ostringstream o;
    o << "{\"version\": " << kTuneFileVersion << ", \"arch\": \"" << arch_ << "\", \"runtime\": " << runtime_
      << ", \"entries\": [\n";
    size_t i = 0;
    for (auto &kv : entries_) {
        o << to_json(kv.second) << (++i < entries_.size() ? ",\n" : "\n");
    }
    o << "]}\n";
    return o.str();
}

bool Tuner::save() const {
    if (path_.empty()) return false;
    const std::string tmp = path_ + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return false;
        out << describe();
        if (!out) return false;
    }
    return std::rename(tmp.c_str(), path_.c_str()) == 0;
}

int choose(int n, const double *ms, const int *melded_lo, const int *melded_hi, double mixed_lo,
           double mixed_hi, double theta, double tie) {
    if (n <= 0) return -1;
    int best = 0;
    for (int i = 1; i < n; ++i)
        if (ms[i] < ms[best]) best = i;
    const int want_lo = mixed_lo >= theta ? 1 : 0;
    const int want_hi = mixed_hi >= theta ? 1 : 0;
    auto agree = [&](int i) { return (melded_lo[i] == want_lo) + (melded_hi[i] == want_hi); };
    int pick = best;
    for (int i = 0; i < n; ++i) {
        if (ms[i] > ms[best] * (1.0 + tie)) continue;
        if (agree(i) > agree(pick) || (agree(i) == agree(pick) && ms[i] < ms[pick])) pick = i;
    }
    return pick;
}

}  // namespace meld
