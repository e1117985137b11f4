// Schedule autotuner cache: key format and lookup (host code).
#pragma once

#include <cstdint>
#include <map>
#include <string>

namespace fdmt {

// Cache key of a workload: "<arch>/nf<Nf>/nd<Nd>/band<f_min>-<f_max>[/gamma<g>]/<in>-><acc>/nt<2^k>",
// numbers printed as by printf's %.6g, 2^k the smallest power of two >= Nt,
// the gamma part only for a delay law other than -2, and "/twoC" after the
// band part for the two-C table rule.
std::string tune_key(const std::string &arch, int nf, int64_t nt, int nd, double f_min, double f_max,
                     int in_dtype, int acc_dtype, double gamma, int rule = 0);

// Reads the cache file at `path` and, when it holds `key`, returns that
// entry's "options" object in `options` with found = true. A missing file is
// an empty cache (found = false, no error); a malformed one returns the
// reason.
std::string tune_lookup(const std::string &path, const std::string &key, std::map<std::string, double> &options,
                        bool &found);

}  // namespace fdmt
