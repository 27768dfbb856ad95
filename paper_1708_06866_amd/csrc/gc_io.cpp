// gc_io.cpp -- edge-file ingestion (host code): the two formats the paper's
// data are distributed in (Sec. II), turned into the 0-based int32 pairs
// gc_build_csr takes.
//
//   TSV   one edge per line, "u <TAB> v <TAB> w" with ids 1..n (w, the
//         weight, is ignored: every edge weighs 1); blank lines and lines
//         starting with '#' or '%' are skipped; any run of spaces or tabs
//         separates fields; "\r\n" line ends are accepted.
//   MMIO  Matrix Market coordinate format: the "%%MatrixMarket matrix
//         coordinate <field> <symmetry>" banner (field pattern, integer or
//         real; symmetry general, symmetric or skew-symmetric), '%' comment
//         lines, the size line "rows cols nnz", then nnz lines "i j [value]"
//         with 1-based indices.  n = max(rows, cols).
//
// The file is memory-mapped and cut into chunks at line ends; one thread per
// chunk counts its data lines, a prefix sum gives every chunk its output
// offset, and the threads parse their lines in place.  Reading is not part
// of the timed path (Sec. IV-B excludes it).
#include <fcntl.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "gc.h"

namespace gc {
void set_error(const std::string &msg);
void clear_error();
}  // namespace gc

using gc::set_error;

namespace {

struct Mapped {
  const char *p = nullptr;
  size_t n = 0;
  int fd = -1;
  ~Mapped() {
    if (p && n) munmap(const_cast<char *>(p), n);
    if (fd >= 0) close(fd);
  }
};

inline bool is_space(char c) { return c == ' ' || c == '\t' || c == '\r'; }

// Parse an unsigned decimal integer at s (after optional blanks); returns the
// position after it, or nullptr if there is none.  Values above 2^62 saturate.
inline const char *parse_u64(const char *s, const char *end, uint64_t *out) {
  while (s < end && is_space(*s)) ++s;
  if (s < end && *s == '+') ++s;
  if (s >= end || *s < '0' || *s > '9') return nullptr;
  uint64_t v = 0;
  while (s < end && *s >= '0' && *s <= '9') {
    if (v < (1ull << 62)) v = v * 10 + (uint64_t)(*s - '0');
    ++s;
  }
  *out = v;
  return s;
}

// A line is data unless it is blank or a comment.
inline bool data_line(const char *s, const char *e) {
  while (s < e && is_space(*s)) ++s;
  return s < e && *s != '#' && *s != '%';
}

const char *line_end(const char *s, const char *end) {
  const void *q = memchr(s, '\n', (size_t)(end - s));
  return q ? static_cast<const char *>(q) : end;
}

// Chunk boundaries at line starts.
std::vector<const char *> chunks(const char *b, const char *e, int parts) {
  std::vector<const char *> cut{b};
  const size_t len = (size_t)(e - b);
  for (int i = 1; i < parts; ++i) {
    const char *q = b + len * i / parts;
    if (q <= cut.back()) continue;
    q = line_end(q, e);
    if (q < e) ++q;
    if (q > cut.back() && q < e) cut.push_back(q);
  }
  cut.push_back(e);
  return cut;
}

// Run fn(i) for every chunk i < nc: chunk 0 on the calling thread, the others
// on threads of their own.  A thread that cannot start (too many threads, no
// address space for its stack) leaves its chunk to the calling thread.
template <class F>
void run_chunks(int nc, F &&fn) {
  std::vector<std::thread> th;
  int started = 1;  // chunks [1, started) run on threads
  try {
    th.reserve((size_t)std::max(nc - 1, 0));
    for (int i = 1; i < nc; ++i) {
      th.emplace_back(fn, i);
      started = i + 1;
    }
  } catch (const std::exception &) {
  }
  for (int i = started; i < nc; ++i) fn(i);
  if (nc > 0) fn(0);
  for (auto &t : th) t.join();
}

struct ChunkOut {
  int64_t lines = 0;
  uint64_t max_id = 0;
  gc_status st = GC_OK;
  int64_t bad_line = -1;  // offset in the file of the first bad line
};

}  // namespace

static gc_status read_edges(const char *path, int32_t format, int32_t *h_src, int32_t *h_dst,
                            int64_t cap, int64_t *n_pairs, int64_t *n_vertices) {
  if (!path || !n_pairs || (format != GC_FILE_AUTO && format != GC_FILE_TSV &&
                            format != GC_FILE_MMIO) ||
      ((h_src == nullptr) != (h_dst == nullptr))) {
    set_error("gc_read_edges: invalid argument");
    return GC_EINVAL;
  }
  Mapped f;
  f.fd = open(path, O_RDONLY);
  if (f.fd < 0) {
    set_error(std::string("gc_read_edges: cannot open ") + path);
    return GC_EINVAL;
  }
  struct stat sb;
  if (fstat(f.fd, &sb) != 0) {
    set_error(std::string("gc_read_edges: cannot stat ") + path);
    return GC_EINVAL;
  }
  f.n = (size_t)sb.st_size;
  const char *b = "";
  if (f.n > 0) {
    void *m = mmap(nullptr, f.n, PROT_READ, MAP_PRIVATE, f.fd, 0);
    if (m == MAP_FAILED) {
      f.n = 0;
      set_error(std::string("gc_read_edges: cannot map ") + path);
      return GC_EINVAL;
    }
    f.p = static_cast<const char *>(m);
    b = f.p;
  }
  const char *e = b + f.n;

  // ---- format, header ----
  const bool banner = f.n >= 14 && memcmp(b, "%%MatrixMarket", 14) == 0;
  const bool mmio = format == GC_FILE_MMIO || (format == GC_FILE_AUTO && banner);
  const char *data = b;
  uint64_t mm_rows = 0, mm_cols = 0, mm_nnz = 0;
  if (mmio) {
    if (!banner) {
      set_error("gc_read_edges: no %%MatrixMarket banner");
      return GC_EINVAL;
    }
    const char *le = line_end(b, e);
    std::string ban(b, le);
    for (char &c : ban) c = (char)tolower((unsigned char)c);
    if (ban.find("coordinate") == std::string::npos ||
        ban.find("complex") != std::string::npos || ban.find("hermitian") != std::string::npos) {
      set_error("gc_read_edges: only coordinate pattern/integer/real matrices are edge lists");
      return GC_EINVAL;
    }
    const char *s = le < e ? le + 1 : e;
    // comments, then the size line
    for (;;) {
      if (s >= e) {
        set_error("gc_read_edges: Matrix Market file without a size line");
        return GC_EINVAL;
      }
      const char *l = line_end(s, e);
      if (data_line(s, l)) {
        const char *q = parse_u64(s, l, &mm_rows);
        if (q) q = parse_u64(q, l, &mm_cols);
        if (q) q = parse_u64(q, l, &mm_nnz);
        if (!q) {
          set_error("gc_read_edges: bad Matrix Market size line");
          return GC_EINVAL;
        }
        data = l < e ? l + 1 : e;
        break;
      }
      s = l < e ? l + 1 : e;
    }
    if (std::max(mm_rows, mm_cols) > (uint64_t)INT32_MAX) {
      set_error("gc_read_edges: more than 2^31 - 1 vertices");
      return GC_EOVERFLOW;
    }
  }

  // ---- pass 1: data lines per chunk ----
  int threads = (int)std::thread::hardware_concurrency();
  threads = std::max(1, std::min(threads, 16));
  if (e - data < (1 << 20)) threads = 1;
  const std::vector<const char *> cut = chunks(data, e, threads);
  const int nc = (int)cut.size() - 1;
  std::vector<ChunkOut> co(nc);
  auto count = [&](int i) {
    int64_t k = 0;
    for (const char *s = cut[i]; s < cut[i + 1];) {
      const char *l = line_end(s, cut[i + 1]);
      k += data_line(s, l);
      s = l < cut[i + 1] ? l + 1 : cut[i + 1];
    }
    co[i].lines = k;
  };
  run_chunks(nc, count);
  std::vector<int64_t> off(nc + 1, 0);
  for (int i = 0; i < nc; ++i) off[i + 1] = off[i] + co[i].lines;
  const int64_t total = off[nc];
  *n_pairs = total;
  if (mmio && (uint64_t)total != mm_nnz) {
    set_error("gc_read_edges: Matrix Market entry count differs from the size line");
    return GC_EINVAL;
  }
  if (n_vertices) *n_vertices = mmio ? (int64_t)std::max(mm_rows, mm_cols) : -1;
  if (!h_src) return GC_OK;  // sizes only
  if (cap < total) {
    set_error("gc_read_edges: cap < number of edges");
    return GC_ECAPACITY;
  }

  // ---- pass 2: parse ----
  const uint64_t id_lim = mmio ? std::max(mm_rows, mm_cols) : (uint64_t)INT32_MAX;
  auto parse = [&](int i) {
    int64_t k = off[i];
    uint64_t mx = 0;
    for (const char *s = cut[i]; s < cut[i + 1];) {
      const char *l = line_end(s, cut[i + 1]);
      if (data_line(s, l)) {
        uint64_t u = 0, v = 0;
        const char *q = parse_u64(s, l, &u);
        if (q) q = parse_u64(q, l, &v);
        // after the two ids: nothing, or blanks and a value field
        if (q && q < l && !is_space(*q)) q = nullptr;
        if (!q) {
          co[i].st = GC_EINVAL;
          co[i].bad_line = s - b;
          return;
        }
        if (u == 0 || v == 0 || u > id_lim || v > id_lim) {
          co[i].st = (u > (uint64_t)INT32_MAX || v > (uint64_t)INT32_MAX) && !mmio ? GC_EOVERFLOW
                                                                                  : GC_ERANGE;
          co[i].bad_line = s - b;
          return;
        }
        h_src[k] = (int32_t)(u - 1);
        h_dst[k] = (int32_t)(v - 1);
        mx = std::max(mx, std::max(u, v));
        ++k;
      }
      s = l < cut[i + 1] ? l + 1 : cut[i + 1];
    }
    co[i].max_id = mx;
  };
  run_chunks(nc, parse);
  uint64_t mx = 0;
  for (int i = 0; i < nc; ++i) {
    if (co[i].st != GC_OK) {
      const char *s = b + co[i].bad_line;
      std::string line(s, line_end(s, e));
      if (line.size() > 80) line.resize(80);
      set_error(std::string(co[i].st == GC_EINVAL ? "gc_read_edges: malformed line: "
                                                  : "gc_read_edges: vertex id out of range: ") +
                line);
      return co[i].st;
    }
    mx = std::max(mx, co[i].max_id);
  }
  if (n_vertices) *n_vertices = mmio ? (int64_t)std::max(mm_rows, mm_cols) : (int64_t)mx;
  return GC_OK;
}

extern "C" gc_status gc_read_edges(const char *path, int32_t format, int32_t *h_src,
                                   int32_t *h_dst, int64_t cap, int64_t *n_pairs,
                                   int64_t *n_vertices) {
  gc::clear_error();
  // no C++ exception may cross the C ABI: a failed host allocation becomes a
  // status (threads that cannot start are handled inside, by run_chunks)
  try {
    return read_edges(path, format, h_src, h_dst, cap, n_pairs, n_vertices);
  } catch (const std::exception &e) {
    try {
      set_error(std::string("gc_read_edges: host allocation failed: ") + e.what());
    } catch (...) {
    }
  } catch (...) {
    try {
      set_error("gc_read_edges: unknown exception");
    } catch (...) {
    }
  }
  return GC_ENOMEM;
}
