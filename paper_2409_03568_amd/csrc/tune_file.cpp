// Persistent autotuning results (text file, one line per device and ring shape).
#include "tune_file.hpp"

#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <unistd.h>

#include <atomic>
#include <fstream>
#include <sstream>
#include <vector>

namespace ckks::tune {

static const char kTag[] = "ckks-tune-v1";

std::string format_line(const Key &k, const Values &v) {
  std::ostringstream os;
  os << kTag << " arch=" << k.arch << " cus=" << k.cus << " log_n=" << k.log_n << " L=" << k.L << " enc=" << v.enc
     << " dec=" << v.dec << " mul=" << v.mul << " row=" << v.row << " gather=" << v.gather;
  return os.str();
}

static bool parse_int(const std::string &s, int *out) {
  if (s.empty() || s.size() > 9) return false;
  int x = 0;
  for (char c : s) {
    if (c < '0' || c > '9') return false;
    x = 10 * x + (c - '0');
  }
  *out = x;
  return true;
}

bool parse_line(const std::string &line, Key *k, Values *v) {
  std::istringstream is(line);
  std::string tok;
  if (!(is >> tok) || tok != kTag) return false;
  Key kk;
  Values vv;
  unsigned seen = 0;
  while (is >> tok) {
    const size_t eq = tok.find('=');
    if (eq == std::string::npos || eq == 0) return false;
    const std::string name = tok.substr(0, eq), val = tok.substr(eq + 1);
    static const char *const kInts[] = {"cus", "log_n", "L", "enc", "dec", "mul", "row", "gather"};
    int *const dst[] = {&kk.cus, &kk.log_n, &kk.L, &vv.enc, &vv.dec, &vv.mul, &vv.row, &vv.gather};
    if (name == "arch") {
      if (val.empty()) return false;
      kk.arch = val;
      seen |= 1u;
      continue;
    }
    bool known = false;
    for (int i = 0; i < 8; i++)
      if (name == kInts[i]) {
        if (!parse_int(val, dst[i])) return false;
        seen |= 2u << i;
        known = true;
      }
    if (!known) return false;
  }
  if (seen != 0x1ffu) return false;
  *k = kk;
  *v = vv;
  return true;
}

static bool width_ok(int w, int log_n) {
  return (w == 8 || w == 16 || w == 32) && ((1 << log_n) / w) <= 1024 && ((1 << log_n) / w) >= 64;
}

bool valid(const Values &v, int log_n) {
  return log_n >= 11 && log_n <= 14 && width_ok(v.enc, log_n) && width_ok(v.dec, log_n) &&
         width_ok(v.mul, log_n) && v.row >= 0 && v.row <= 64 && v.gather >= 1 && v.gather <= 64;
}

static int read_lines(const char *path, std::vector<std::string> *lines, bool *exists) {
  errno = 0;
  std::ifstream f(path);
  *exists = false;
  if (!f) {
    if (errno == ENOENT) return 0;
    return errno ? errno : EIO;
  }
  *exists = true;
  std::string line;
  while (std::getline(f, line)) lines->push_back(line);
  if (f.bad()) return EIO;
  return 0;
}

int store(const char *path, const Key &k, const Values &v) {
  if (!path || !*path) return EINVAL;
  std::vector<std::string> lines;
  bool exists = false;
  if (int e = read_lines(path, &lines, &exists)) return e;
  std::vector<std::string> keep;
  for (const std::string &l : lines) {
    Key lk;
    Values lv;
    if (parse_line(l, &lk, &lv) && lk == k) continue;
    keep.push_back(l);
  }
  keep.push_back(format_line(k, v));
  // a temporary name of this process and call, so concurrent stores never share one
  static std::atomic<unsigned> serial{0};
  const std::string tmp =
      std::string(path) + ".tmp" + std::to_string((long)getpid()) + "." + std::to_string(serial.fetch_add(1));
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return errno ? errno : EIO;
  bool ok = true;
  for (const std::string &l : keep) ok = ok && fprintf(f, "%s\n", l.c_str()) >= 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok) {
    (void)remove(tmp.c_str());
    return EIO;
  }
  if (rename(tmp.c_str(), path) != 0) {
    const int e = errno ? errno : EIO;
    (void)remove(tmp.c_str());
    return e;
  }
  return 0;
}

int lookup(const char *path, const Key &k, Values *v, bool *found) {
  *found = false;
  if (!path || !*path) return EINVAL;
  std::vector<std::string> lines;
  bool exists = false;
  if (int e = read_lines(path, &lines, &exists)) return e;
  for (const std::string &l : lines) {
    Key lk;
    Values lv;
    if (parse_line(l, &lk, &lv) && lk == k) {
      *v = lv;
      *found = true;
    }
  }
  return 0;
}

}  // namespace ckks::tune
