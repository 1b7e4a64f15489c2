// Persisted choices of the block-product autotuner: a JSON file of entries, each mapping a key
// (architecture, arithmetic, problem count, connection-term count and the sector-dimension
// histogram of the superblock blocks) to the dmrg_gemm bits the autotuner chose and the
// per-family timings it measured.  Host code only.
#pragma once

#include <string>
#include <vector>

namespace dmrg {

struct Plan;

constexpr int kTuneTimes = 10;     // per-family milliseconds stored with an entry
constexpr int kTuneBucket = 16;    // width of the histogram's dimension buckets

struct TuneEntry {
    std::string key;
    int variant = 0;
    double ms[kTuneTimes];         // -1 where not timed
};

// Key of the plans (one per problem of a batch) in arithmetic `precision` on architecture
// `arch`: "<arch>/<arithmetic>/problems=P/terms=T/S=<bucket>:<count>,.../E=...", where S and E
// count the superblock blocks whose system (environment) sector dimension rounds up to each
// multiple of kTuneBucket.
std::string tune_key(const std::vector<const Plan*>& plans, int precision, const std::string& arch);

// Reads every entry of the cache at path.  A missing file is an empty cache.  Returns an empty
// string on success, else the reason the file cannot be used (unreadable, not JSON, not a cache
// of this format).
std::string tune_cache_read(const std::string& path, std::vector<TuneEntry>& out);

// Finds key; found = false when the file or the key is absent.  Returns the reason on error.
std::string tune_cache_find(const std::string& path, const std::string& key, TuneEntry& out,
                            bool& found);

// Stores one entry (replacing an entry of the same key): the file is read, updated and written
// to a temporary file in the same directory (path.tmp.<pid>.<n>, n counting this process's
// stores) that is then renamed over it, so readers never see a partial file.  Writers that
// overlap may drop each other's new entries (the lost key is timed again on its next lookup).
// Returns the reason on error.
std::string tune_cache_put(const std::string& path, const TuneEntry& e);

}  // namespace dmrg
