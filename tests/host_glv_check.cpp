// Drives the library's host G1 scalar multiplication by the G1 endomorphism
// (host_field.hpp) for test_host_glv.py.  Each input line holds, in hex,
// px py qx qy k b (affine P and Q, scalars k and b below r); each output line
// holds the affine k P (sum of the two GLV halves), the affine k P + b Q
// (one shared chain), and the split of k: sign and magnitude of k1 and k2.
#include <cstdio>
#include <cstring>
#include <iostream>
#include <string>

#include "host_field.hpp"

using namespace zkvc::host;

static void parse(const std::string& hex, uint64_t w[4]) {
  std::memset(w, 0, 4 * sizeof(uint64_t));
  int bit = 0;
  for (int i = (int)hex.size() - 1; i >= 0; i--, bit += 4) {
    const char c = hex[i];
    const uint64_t v = c <= '9' ? c - '0' : (c | 32) - 'a' + 10;
    w[bit / 64] |= v << (bit % 64);
  }
}

static void print_words(const uint64_t w[4]) {
  std::printf("%016llx%016llx%016llx%016llx", (unsigned long long)w[3], (unsigned long long)w[2],
              (unsigned long long)w[1], (unsigned long long)w[0]);
}

static void print_point(const G1J& p) {
  if (p.is_inf()) {
    std::printf("inf inf");
    return;
  }
  HFq x, y;
  p.to_affine(x, y);
  uint64_t w[4];
  x.to_u64(w);
  print_words(w);
  std::printf(" ");
  y.to_u64(w);
  print_words(w);
}

int main() {
  std::string px, py, qx, qy, ks, bs;
  while (std::cin >> px >> py >> qx >> qy >> ks >> bs) {
    uint64_t w[4], k[4], b[4];
    parse(px, w);
    const HFq x1 = HFq::from_u64(w);
    parse(py, w);
    const G1J P = G1J::from_affine(x1, HFq::from_u64(w));
    parse(qx, w);
    const HFq x2 = HFq::from_u64(w);
    parse(qy, w);
    const G1J Q = G1J::from_affine(x2, HFq::from_u64(w));
    parse(ks, k);
    parse(bs, b);
    const GlvSplit s = glv_split(k);
    print_point(G1J::add(glv_half(P, s, 0), glv_half(P, s, 1)));
    std::printf(" ");
    print_point(glv_mul2(P, k, Q, b));
    for (int h = 0; h < 2; h++) {
      std::printf(" %d ", (int)s.neg[h]);
      print_words(s.mag[h]);
    }
    std::printf("\n");
  }
  return 0;
}
