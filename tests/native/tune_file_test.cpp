// CPU test of the tuning-file module (format, parse, validation, merge, lookup), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers_cpu.py.
// argv[1] is a scratch directory.  Prints "OK".
#include <stdio.h>
#include <stdlib.h>

#include <fstream>
#include <string>

#include "../../paper_2409_03568_amd/csrc/tune_file.hpp"

using namespace ckks::tune;

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__); \
      exit(1);                                                 \
    }                                                          \
  } while (0)

static int count_lines(const std::string &path) {
  std::ifstream f(path);
  std::string l;
  int n = 0;
  while (std::getline(f, l)) n++;
  return n;
}

int main(int argc, char **argv) {
  CHECK(argc == 2);
  const std::string dir = argv[1];
  Key k{"gfx950:sramecc+:xnack-", 256, 13, 3};
  Values v{8, 16, 32, 4, 8};
  Key k2;
  Values v2;
  // round trip
  CHECK(parse_line(format_line(k, v), &k2, &v2));
  CHECK(k2 == k && v2.enc == 8 && v2.dec == 16 && v2.mul == 32 && v2.row == 4 && v2.gather == 8);
  // malformed lines
  const char *bad[] = {"", "ckks-tune-v1", "ckks-tune-v2 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=8",
                       "ckks-tune-v1 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0",
                       "ckks-tune-v1 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=x",
                       "ckks-tune-v1 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=-1 gather=8",
                       "ckks-tune-v1 arch= cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=8",
                       "ckks-tune-v1 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=8 extra=1",
                       "ckks-tune-v1 arch=a cus=1 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=99999999999",
                       "ckks-tune-v1 arch=a cus=1 =2 log_n=13 L=3 enc=8 dec=8 mul=8 row=0 gather=8"};
  for (const char *b : bad) CHECK(!parse_line(b, &k2, &v2));
  // validation
  CHECK(valid(v, 13));
  CHECK(!valid(Values{8, 8, 8, 0, 8}, 14));   // 2048 threads
  CHECK(valid(Values{32, 32, 32, 0, 8}, 11)); // 64 threads
  CHECK(!valid(Values{12, 8, 8, 0, 8}, 13));
  CHECK(!valid(Values{8, 8, 8, 65, 8}, 13));
  CHECK(!valid(Values{8, 8, 8, 0, 0}, 13));
  CHECK(!valid(v, 15));
  // missing file
  const std::string path = dir + "/tune.txt";
  bool found = true;
  CHECK(lookup(path.c_str(), k, &v2, &found) == 0 && !found);
  // merge keeps foreign lines, replaces the matching one
  {
    std::ofstream f(path);
    f << "# comment line\n" << format_line(Key{"gfx942", 304, 13, 3}, Values{16, 16, 16, 0, 8}) << "\n";
  }
  CHECK(store(path.c_str(), k, v) == 0);
  CHECK(count_lines(path) == 3);
  Values v3{16, 8, 8, 0, 2};
  CHECK(store(path.c_str(), k, v3) == 0);
  CHECK(count_lines(path) == 3);
  CHECK(lookup(path.c_str(), k, &v2, &found) == 0 && found && v2.enc == 16 && v2.gather == 2);
  CHECK(lookup(path.c_str(), Key{"gfx942", 304, 13, 3}, &v2, &found) == 0 && found && v2.enc == 16);
  CHECK(lookup(path.c_str(), Key{"gfx950:sramecc+:xnack-", 256, 13, 4}, &v2, &found) == 0 && !found);
  // the last matching line wins
  {
    std::ofstream f(path, std::ios::app);
    f << format_line(k, Values{32, 32, 32, 16, 32}) << "\n";
  }
  CHECK(lookup(path.c_str(), k, &v2, &found) == 0 && found && v2.enc == 32 && v2.row == 16);
  // a directory is not a writable file
  CHECK(store(dir.c_str(), k, v) != 0);
  CHECK(store("", k, v) != 0 && lookup(nullptr, k, &v2, &found) != 0);
  printf("OK\n");
  return 0;
}
