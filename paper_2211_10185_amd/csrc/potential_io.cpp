// Host-only part of the C ABI: complex potentials from and to ASCII files
// (Sec. 1: arbitrary complex potentials loaded from ASCII files of numbers).
// No device code; built into the library and, on its own, under host sanitizers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "qfdtd.h"

// message of the last failing context-free call on this thread (qfdtd_last_error(NULL))
thread_local std::string g_create_error;

namespace {
qfdtd_status io_fail(const std::string &msg) {
  g_create_error = msg;
  return QFDTD_E_INVALID;
}
}  // namespace

extern "C" {

// ASCII potential files.  Records are lines; '#' starts a comment; fields are separated by
// blanks, tabs or commas.  Every record has the same number of fields:
//   1: re            2: re im          (N^3 records in C order, x3 fastest)
//   4: i1 i2 i3 re   5: i1 i2 i3 re im (every site exactly once, any order)
qfdtd_status qfdtd_read_potential_ascii(const char *path, int32_t N, double *grid) {
  if (!path || !grid) return io_fail("NULL argument");
  if (N < 1 || N > 1024) return io_fail("N must be 1..1024");
  FILE *f = std::fopen(path, "rb");
  if (!f) return io_fail(std::string("cannot open ") + path);
  std::string text;
  {
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
  }
  const size_t n3 = (size_t)N * N * N;
  std::vector<unsigned char> seen;
  int fields = -1;
  size_t rec = 0, line_no = 0, pos = 0;
  double v[6];
  std::string line;
  while (pos < text.size()) {
    size_t end = text.find('\n', pos);
    if (end == std::string::npos) end = text.size();
    ++line_no;
    line.assign(text, pos, end - pos);
    pos = end + 1;
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    for (char &ch : line)
      if (ch == ',' || ch == '\t' || ch == '\r') ch = ' ';
    int nf = 0;
    const char *p = line.c_str();
    while (true) {
      while (*p == ' ') ++p;
      if (!*p) break;
      char *q = nullptr;
      const double x = std::strtod(p, &q);
      if (q == p || nf == 6) return io_fail("bad number or too many fields on line " + std::to_string(line_no));
      v[nf++] = x;
      p = q;
    }
    if (nf == 0) continue;
    if (fields < 0) {
      if (nf != 1 && nf != 2 && nf != 4 && nf != 5)
        return io_fail("records need 1, 2, 4 or 5 fields (line " + std::to_string(line_no) + ")");
      fields = nf;
      for (size_t g = 0; g < 2 * n3; ++g) grid[g] = 0.0;
      if (fields >= 4) seen.assign(n3, 0);
    } else if (nf != fields) {
      return io_fail("inconsistent field count on line " + std::to_string(line_no));
    }
    size_t g;
    int o = 0;
    if (fields >= 4) {
      long long ii[3];
      for (int a = 0; a < 3; ++a) {
        if (v[a] != std::floor(v[a]) || v[a] < 0 || v[a] >= N)
          return io_fail("site index out of range on line " + std::to_string(line_no));
        ii[a] = (long long)v[a];
      }
      g = ((size_t)ii[0] * N + (size_t)ii[1]) * N + (size_t)ii[2];
      if (seen[g]) return io_fail("site given twice (line " + std::to_string(line_no) + ")");
      seen[g] = 1;
      o = 3;
    } else {
      if (rec >= n3) return io_fail("more than N^3 records");
      g = rec;
    }
    if (!std::isfinite(v[o]))
      return io_fail("non-finite value on line " + std::to_string(line_no));
    grid[2 * g] = v[o];
    grid[2 * g + 1] = (fields == 2 || fields == 5) ? v[o + 1] : 0.0;
    if (!std::isfinite(grid[2 * g + 1])) return io_fail("non-finite value on line " + std::to_string(line_no));
    ++rec;
  }
  if (fields < 0) return io_fail("no records");
  if (rec != n3) return io_fail("expected N^3 = " + std::to_string(n3) + " records, found " + std::to_string(rec));
  return QFDTD_OK;
}

qfdtd_status qfdtd_write_potential_ascii(const char *path, int32_t N, const double *grid) {
  if (!path || !grid) return io_fail("NULL argument");
  if (N < 1 || N > 1024) return io_fail("N must be 1..1024");
  FILE *f = std::fopen(path, "wb");
  if (!f) return io_fail(std::string("cannot create ") + path);
  std::fprintf(f, "# complex potential on a %d^3 lattice: re im per site, C order (x3 fastest)\n", N);
  const size_t n3 = (size_t)N * N * N;
  bool ok = true;
  for (size_t g = 0; g < n3 && ok; ++g) ok = std::fprintf(f, "%.17g %.17g\n", grid[2 * g], grid[2 * g + 1]) > 0;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? QFDTD_OK : io_fail(std::string("write failed: ") + path);
}

}  // extern "C"
