// Persistent autotuning results: one text line per (device architecture, compute units,
// ring degree, number of primes), so a process can reuse the register blocking and launch
// shapes a previous one measured instead of timing them again.  Plain C++ (no HIP), so the
// parser and the file merge are tested on the CPU under the sanitizers.
//
// Line format (fields separated by single spaces, any order after the tag):
//   ckks-tune-v1 arch=gfx950:sramecc+:xnack- cus=256 log_n=13 L=3 enc=8 dec=8 mul=16 row=0 gather=8
// enc, dec, mul: values per thread of the encryption, decryption and product kernels;
// row: workgroups per compute unit of the row-wise kernels (0: one workgroup per row);
// gather: workgroups per compute unit of the value-cache gather.  Lines that do not parse
// are kept as they are by a merge and ignored by a lookup.
#pragma once

#include <string>

namespace ckks::tune {

struct Key {
  std::string arch;
  int cus = 0, log_n = 0, L = 0;
  bool operator==(const Key &o) const { return arch == o.arch && cus == o.cus && log_n == o.log_n && L == o.L; }
};

struct Values {
  int enc = 0, dec = 0, mul = 0;  // values per thread
  int row = 0, gather = 0;        // workgroups per compute unit
};

// The line for (k, v), without a newline.
std::string format_line(const Key &k, const Values &v);
// Parses one line; false if it is not a complete, well-formed tuning line.
bool parse_line(const std::string &line, Key *k, Values *v);
// True when v holds settings the kernels support for ring degree 2^log_n.
bool valid(const Values &v, int log_n);
// Writes (k, v) into the file at path: replaces the line with the same key, or appends
// one; other lines are kept.  The new contents go to a temporary file that is renamed
// over the old one, so a reader sees the old file or the new one.  0 on success, else an
// errno value.
int store(const char *path, const Key &k, const Values &v);
// Looks up k in the file at path: 0 with *found set (and *v filled when found); a missing
// file is found = false, other read errors return their errno value.  The last matching
// line wins.
int lookup(const char *path, const Key &k, Values *v, bool *found);

}  // namespace ckks::tune
