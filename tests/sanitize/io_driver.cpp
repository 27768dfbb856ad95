// Runs gc_read_edges (paper_1708_06866_amd/csrc/gc_io.cpp, host code) under
// AddressSanitizer and UndefinedBehaviorSanitizer on the files named on the
// command line: each argument is "<expect>:<path>", where <expect> is the
// status the read must return ("0" = GC_OK, then the pairs are printed as
// "u v" lines for the test to compare) or a negative status.  Built by
// tests/test_sanitize.py; test infrastructure.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "gc.h"

// gc_io.cpp reports failures through the library's error text; the driver
// keeps the last one to print it.
namespace gc {
static std::string last;
void set_error(const std::string &msg) { last = msg; }
void clear_error() { last.clear(); }
}  // namespace gc

int main(int argc, char **argv) {
  int bad = 0;
  for (int i = 1; i < argc; ++i) {
    std::string arg = argv[i];
    const size_t colon = arg.find(':');
    const int expect = std::atoi(arg.substr(0, colon).c_str());
    const std::string path = arg.substr(colon + 1);
    int64_t np = 0, nv = 0;
    gc_status st = gc_read_edges(path.c_str(), GC_FILE_AUTO, nullptr, nullptr, 0, &np, &nv);
    std::vector<int32_t> s, d;
    if (st == GC_OK) {
      s.resize((size_t)np + 1);
      d.resize((size_t)np + 1);
      st = gc_read_edges(path.c_str(), GC_FILE_AUTO, s.data(), d.data(), np, &np, &nv);
    }
    if (st != expect) {
      std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", path.c_str(), st, expect,
                   gc::last.c_str());
      ++bad;
      continue;
    }
    std::printf("# %s %lld %lld\n", path.c_str(), (long long)np, (long long)nv);
    if (st == GC_OK)
      for (int64_t k = 0; k < np; ++k) std::printf("%d %d\n", s[k], d[k]);
  }
  return bad ? 1 : 0;
}
