// Drives the library's host-only code (paper_1605_08423_amd/csrc/host.cpp: the Hueckel
// eigen-solver, the reciprocal-vector builder, the admission rule and the checkpoint
// validation) with valid, edge-case and damaged inputs, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure).  Exit 0 when every call returns as
// expected; the sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "host.hpp"

#define EXPECT(c)                                               \
  do {                                                          \
    if (!(c)) {                                                 \
      std::printf("FAILED %s at line %d\n", #c, __LINE__);      \
      return 1;                                                 \
    }                                                           \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  // Hueckel orbitals on random boxes, every twist
  for (int n : {2, 4, 16, 54}) {
    const double L = 1.4 * std::cbrt(4.18879 * n);
    std::vector<double> R(3 * n), z(n), C((size_t)n * (n / 2));
    for (double& x : R) x = L * U(rng);
    for (double& x : z) x = 0.8 + 0.4 * U(rng);
    for (int tw = 0; tw < 8; ++tw) {
      EXPECT(vmc_huckel_params_twist(n, L, tw, R.data(), z.data(), C.data()) == VMC_OK);
      for (double c : C) EXPECT(std::isfinite(c));
    }
    EXPECT(vmc_huckel_params_twist(n, L, 8, R.data(), z.data(), C.data()) == VMC_EINVAL);
    std::vector<double> Rbad = R;
    Rbad[1] = std::numeric_limits<double>::quiet_NaN();
    EXPECT(vmc_huckel_params(n, L, Rbad.data(), z.data(), C.data()) == VMC_EINVAL);
    std::vector<double> zbad = z;
    zbad[0] = 0.0;
    EXPECT(vmc_huckel_params(n, L, R.data(), zbad.data(), C.data()) == VMC_EINVAL);
  }
  EXPECT(vmc_huckel_params(3, 5.0, nullptr, nullptr, nullptr) == VMC_EINVAL);
  // reciprocal vectors: half of the nonzero lattice points in the ball of radius nmax
  for (int nm = 1; nm <= 12; ++nm) {
    vmc_system s{};
    s.n_protons = 16; s.box_L = 6.0; s.ewald_kappa = 1.3; s.ewald_nmax = nm;
    std::vector<double> kv;
    std::vector<int> slots, nx0;
    vmc_host::build_kvectors(s, kv, slots, nx0);
    int full = 0;
    for (int x = -nm; x <= nm; ++x)
      for (int y = -nm; y <= nm; ++y)
        for (int zz = -nm; zz <= nm; ++zz) full += (x * x + y * y + zz * zz <= nm * nm) ? 1 : 0;
    EXPECT((int)kv.size() / 4 == (full - 1) / 2);
    int tot = 0;
    for (size_t q = 0; q < nx0.size(); ++q) tot += slots[4 * q + 3];
    EXPECT(tot == (int)kv.size() / 4);
  }
  // admission: FIFO without overtaking, no overflow near SIZE_MAX
  const size_t big = std::numeric_limits<size_t>::max();
  const size_t b1[4] = {3, 4, 1, 1};
  EXPECT(vmc_host::admit_count(8, 0, 4, b1) == 3);   // 3 + 4 + 1 = 8 fits, the next does not
  EXPECT(vmc_host::admit_count(8, 2, 4, b1) == 1);   // 2 + 3 + 4 > 8: the small ones wait
  const size_t b2[2] = {big, 1};
  EXPECT(vmc_host::admit_count(big - 1, 0, 2, b2) == 0);
  EXPECT(vmc_host::admit_count(big, 1, 2, b2) == 0);
  EXPECT(vmc_host::admit_count(big, big - 2, 1, b2 + 1) == 1);
  EXPECT(vmc_server_admit_count(10, 0, -1, b1) == -1);
  EXPECT(vmc_server_admit_count(10, 0, 1, nullptr) == -1);
  // checkpoints: a sealed buffer validates; any flipped byte, truncation or foreign buffer does not
  for (int n : {2, 16}) {
    for (int w : {1, 3}) {
      const size_t len = sizeof(vmc_host::CkptHeader) + vmc_host::ckpt_payload_bytes(n, w);
      std::vector<unsigned char> buf(len + 7);
      vmc_host::CkptHeader h;
      vmc_host::ckpt_init_header(&h, n, w);
      h.seed = 7; h.box_L = 5.0;
      std::memcpy(buf.data(), &h, sizeof h);
      for (size_t i = sizeof h; i < buf.size(); ++i) buf[i] = (unsigned char)(rng() & 0xff);
      vmc_host::ckpt_seal(buf.data());
      vmc_host::CkptHeader out;
      EXPECT(vmc_host::ckpt_validate(buf.data(), len, &out) == VMC_OK);
      EXPECT(out.seed == 7 && out.n == n && out.w == w);
      EXPECT(vmc_host::ckpt_validate(buf.data(), len + 7, nullptr) == VMC_OK);   // trailing bytes are ignored
      for (size_t cut : {(size_t)0, (size_t)1, sizeof h - 1, sizeof h, len - 1})
        EXPECT(vmc_host::ckpt_validate(buf.data(), cut, nullptr) == VMC_EINVAL);
      for (int k = 0; k < 300; ++k) {
        const size_t pos = (size_t)(rng() % len);
        const unsigned char bit = (unsigned char)(1u << (rng() % 8));
        buf[pos] ^= bit;
        EXPECT(vmc_host::ckpt_validate(buf.data(), len, nullptr) == VMC_EINVAL);
        buf[pos] ^= bit;
      }
      EXPECT(vmc_host::ckpt_validate(buf.data(), len, nullptr) == VMC_OK);
    }
  }
  // random garbage and headers claiming absurd sizes
  for (int k = 0; k < 200; ++k) {
    std::vector<unsigned char> g(1 + rng() % 4096);
    for (auto& c : g) c = (unsigned char)(rng() & 0xff);
    EXPECT(vmc_host::ckpt_validate(g.data(), g.size(), nullptr) == VMC_EINVAL);
  }
  {
    vmc_host::CkptHeader h;
    vmc_host::ckpt_init_header(&h, 16, 4);
    h.n = 1 << 30;
    EXPECT(vmc_host::ckpt_validate(&h, sizeof h, nullptr) == VMC_EINVAL);
    vmc_host::ckpt_init_header(&h, 16, 4);
    h.w = -5;
    EXPECT(vmc_host::ckpt_validate(&h, sizeof h, nullptr) == VMC_EINVAL);
    EXPECT(vmc_host::ckpt_validate(nullptr, 100, nullptr) == VMC_EINVAL);
  }
  std::printf("host driver ok\n");
  return 0;
}
