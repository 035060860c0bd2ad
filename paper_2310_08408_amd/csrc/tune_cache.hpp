// On-disk records of the autotuner's choices: one text line per tuned
// shape, keyed by (GPU architecture, element size, pass kind, length, lines,
// valid input length, kept output length, batch).  Plain C++ (no HIP), so
// the parser can be exercised on the host, also under sanitizers.
//
// Line format (fields separated by blanks):
//   libprop-tune 1 <arch> <elem_bytes> <kind> <n> <lines> <n_in> <n_out> <batch> <variant>
// A line that does not parse, has another tag or version, or holds a value
// out of range is rejected; the caller additionally checks that the
// variant is a valid candidate of that shape before using it.
#pragma once

#include <cstdint>
#include <cstdio>
#include <sstream>
#include <string>

namespace lp {

struct TuneRecord {
  std::string arch;
  int elem = 0;  // bytes of the real element type: 4 (complex64) or 8 (complex128)
  int kind = 0, n = 0, lines = 0, n_in = 0, n_out = 0, batch = 0, variant = 0;
};

constexpr int kTuneKinds = 4;      // RS columns, vectorial mixing, Bluestein columns, Bluestein rows
constexpr int kTuneCandidates = 6;  // lines variants x schedules

inline std::string format_tune_record(const TuneRecord& r) {
  std::ostringstream o;
  o << "libprop-tune 1 " << r.arch << ' ' << r.elem << ' ' << r.kind << ' ' << r.n << ' ' << r.lines << ' '
    << r.n_in << ' ' << r.n_out << ' ' << r.batch << ' ' << r.variant;
  return o.str();
}

// true and *out filled if `line` is a well-formed record with values in range
inline bool parse_tune_record(const std::string& line, TuneRecord* out) {
  std::istringstream in(line);
  std::string tag;
  int version = 0;
  TuneRecord r;
  if (!(in >> tag >> version >> r.arch >> r.elem >> r.kind >> r.n >> r.lines >> r.n_in >> r.n_out >> r.batch >>
        r.variant))
    return false;
  std::string extra;
  if (in >> extra) return false;
  if (tag != "libprop-tune" || version != 1) return false;
  if (r.arch.empty() || r.arch.size() > 64) return false;
  for (char ch : r.arch)
    if (!((ch >= 'a' && ch <= 'z') || (ch >= '0' && ch <= '9') || ch == '_' || ch == '-')) return false;
  if (r.elem != 4 && r.elem != 8) return false;
  if (r.kind < 0 || r.kind >= kTuneKinds) return false;
  if (r.n < 1 || r.n > 8192 || r.lines < 1 || r.n_in < 1 || r.n_out < 1 || r.batch < 1) return false;
  if (r.n_in > r.n || r.n_out > r.n) return false;
  if (r.variant < 0 || r.variant >= kTuneCandidates) return false;
  *out = r;
  return true;
}

}  // namespace lp
