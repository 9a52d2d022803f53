// Autotuner state: decisions per (operation, shape class), kept in memory and
// optionally in a JSON file. Host code only.
#pragma once

#include <map>
#include <string>

namespace meld {

struct TuneEntry {
    std::string op;    // "region", "sort", "segsort"
    std::string key;   // shape class
    int lo = 1;        // form of the phases k <= 64 (or of the region): 1 melded, 0 divergent
    int hi = 1;        // form of the phases k >= 128
    int log_t = 0;     // sort tile size (log2), 0 if not applicable
    int xch = 0;       // sorts: phases k <= 64 with lane exchanges (1) or the LDS network (0)
    int form = 0;      // region: 0 divergent, 1 melded, 3 melded with aligned gathers
    double ms = 0;     // median time of the chosen candidate
    double mixed_lo = 0, mixed_hi = 0;  // probe: mixed-wave fraction per stage
    int trials = 0;    // candidates timed
};

class Tuner {
  public:
    // Identity of the machine the decisions were made on; entries from a file
    // with another identity are ignored.
    void set_identity(const std::string &arch, int runtime) {
        arch_ = arch;
        runtime_ = runtime;
    }
    // Loads decisions from path (if it exists and matches) and saves every
    // new decision there. Returns false on a malformed file.
    bool attach(const std::string &path);
    const TuneEntry *find(const std::string &op, const std::string &key) const;
    void put(const TuneEntry &e);  // saves when a file is attached
    std::string describe() const;  // all entries as JSON
    bool save() const;

  private:
    std::map<std::string, TuneEntry> entries_;
    std::string path_;
    std::string arch_;
    int runtime_ = 0;
};

// Index of the chosen candidate: the fastest, unless others are within `tie`
// (relative) of it, in which case the one whose per-stage forms agree most
// with the probe wins (melded for a stage whose mixed-wave fraction is at
// least theta, divergent otherwise).
int choose(int n, const double *ms, const int *melded_lo, const int *melded_hi, double mixed_lo,
           double mixed_hi, double theta, double tie);

}  // namespace meld
