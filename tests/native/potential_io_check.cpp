// Exercises the ASCII potential reader and writer of the C ABI (a host-only source) so
// that they can run under AddressSanitizer and UndefinedBehaviorSanitizer: round trips in
// every record format, boundary inputs and seeded malformed files.  Exit status 0 when
// every check holds; any sanitizer report aborts the run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "qfdtd.h"

static int failures = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);     \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

static void write_text(const std::string &path, const std::string &s) {
  FILE *f = std::fopen(path.c_str(), "wb");
  if (!f) { ++failures; return; }
  std::fwrite(s.data(), 1, s.size(), f);
  std::fclose(f);
}

static std::string num(double x) {
  char b[64];
  std::snprintf(b, sizeof(b), "%.17g", x);
  return b;
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  const std::string path = dir + "/pot.txt";
  std::mt19937_64 rng(20221118);
  std::normal_distribution<double> nd(0.0, 1.0);

  // writer -> reader round trips, values over many magnitudes
  for (int N = 1; N <= 5; ++N) {
    const size_t n3 = (size_t)N * N * N;
    std::vector<double> g(2 * n3), back(2 * n3, -1.0);
    for (size_t i = 0; i < 2 * n3; ++i) g[i] = nd(rng) * std::pow(10.0, (double)((int)(i % 13) - 6) * 25.0);
    CHECK(qfdtd_write_potential_ascii(path.c_str(), N, g.data()) == QFDTD_OK);
    CHECK(qfdtd_read_potential_ascii(path.c_str(), N, back.data()) == QFDTD_OK);
    for (size_t i = 0; i < 2 * n3; ++i) CHECK(back[i] == g[i]);
  }

  // indexed records in shuffled order, with comments, commas and tabs
  {
    const int N = 3;
    std::vector<int> order(27);
    for (int i = 0; i < 27; ++i) order[i] = i;
    std::shuffle(order.begin(), order.end(), rng);
    std::string s = "# indexed\n";
    std::vector<double> want(54);
    for (int i : order) {
      const double re = nd(rng), im = nd(rng);
      want[2 * i] = re;
      want[2 * i + 1] = im;
      s += std::to_string(i / 9) + ",\t" + std::to_string((i / 3) % 3) + " " + std::to_string(i % 3) + " " + num(re) +
           " " + num(im) + "   # site\r\n";
    }
    write_text(path, s);
    std::vector<double> got(54);
    CHECK(qfdtd_read_potential_ascii(path.c_str(), N, got.data()) == QFDTD_OK);
    for (int i = 0; i < 54; ++i) CHECK(got[i] == want[i]);
  }

  // boundary inputs: each must be rejected with QFDTD_E_INVALID, never crash
  const char *bad[] = {"", "\n\n# only comments\n", "1 2 3 4 5 6\n", "1e400 0\n", "nan\n", "0 0 0\n",
                       "0 0 0 1\n0 0 0 1\n", "-1 0 0 1\n", "0.5 0 0 1\n", "1 x\n", "1\n2 3\n"};
  for (const char *b : bad) {
    write_text(path, b);
    std::vector<double> g(16);
    CHECK(qfdtd_read_potential_ascii(path.c_str(), 2, g.data()) == QFDTD_E_INVALID);
  }
  {
    std::string longline(1 << 20, ' ');
    longline += "1.5 2.5\n";
    write_text(path, longline);
    double g[2];
    CHECK(qfdtd_read_potential_ascii(path.c_str(), 1, g) == QFDTD_OK && g[0] == 1.5 && g[1] == 2.5);
  }
  CHECK(qfdtd_read_potential_ascii((dir + "/missing.txt").c_str(), 2, nullptr) == QFDTD_E_INVALID);
  CHECK(qfdtd_read_potential_ascii(nullptr, 2, nullptr) == QFDTD_E_INVALID);

  // seeded malformed files: random bytes and random token soups
  const char alphabet[] = "0123456789+-.eEnaix#, \t\r\n\x01\xff";
  for (int t = 0; t < 400; ++t) {
    std::string s;
    const size_t len = rng() % 600;
    for (size_t i = 0; i < len; ++i) s += (t % 2) ? (char)(rng() % 256) : alphabet[rng() % (sizeof(alphabet) - 1)];
    write_text(path, s);
    const int N = 1 + (int)(rng() % 3);
    std::vector<double> g(2 * N * N * N);
    const qfdtd_status st = qfdtd_read_potential_ascii(path.c_str(), N, g.data());
    CHECK(st == QFDTD_OK || st == QFDTD_E_INVALID);
    if (st == QFDTD_OK)
      for (double x : g) CHECK(std::isfinite(x));
  }

  std::printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
