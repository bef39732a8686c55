// Host-only parts of the library: no HIP types or calls, so they build with a plain C++
// compiler as well (the CPU sanitizer test compiles this file with g++ and
// AddressSanitizer/UndefinedBehaviorSanitizer).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/vmc.h"

namespace vmc_host {

// Half-space reciprocal vectors k = 2 pi n / L, 0 < |n|^2 <= nmax^2, grouped in (ny, nz) slots
// with nx innermost; kv: nk x 4 (kx, ky, kz, W_k = 4 pi / V e^{-k^2/(4 kappa^2)} / k^2); slots:
// nslot x 4 (ny, nz, first k, count), sorted by nx range, longest first; nx0: first nx per slot.
void build_kvectors(const vmc_system& s, std::vector<double>& kv, std::vector<int>& slots, std::vector<int>& nx0);

// Number of queue-head requests admitted, first come first served, while the running
// total stays within the budget.
int admit_count(size_t budget, size_t resident, int n, const size_t* bytes);

// ------------------------------------------------------------ checkpoint --
// Layout: CkptHeader, then the payload in host byte order: walker positions (W x N x 3),
// per-walker means (W x (1 + 9N)), per-walker forces (W x 3N), the last estimate
// [E, sigma_E, acceptance, f] (3 + 3N), the Langevin state R, R_prev (3N each), S, S_prev
// (3N x 3N each) as doubles, then accepted moves (W) as int64.  `checksum` is FNV-1a (64 bit)
// over the header (checksum field zero) and the payload.
struct CkptHeader {
  char magic[8];
  uint32_t version, seed, traj_id, lang_step;
  int32_t n, w, precision, nmax, twist, have_means, have_R, have_prev, have_S, general_twist, contracted, pad_;
  double box_L, kappa, a_par, a_anti, b, j1_b1, theta[3], eta, j3_f[3], j1_f[2];
  uint64_t payload_bytes, checksum;
};
constexpr uint32_t kCkptVersion = 4;
size_t ckpt_payload_bytes(int n, int w);
// Writes magic, version and payload size into h (the caller fills the rest).
void ckpt_init_header(CkptHeader* h, int n, int w);
// Computes and stores the checksum of a buffer holding a header and its payload.
void ckpt_seal(void* buf);
// Checks magic, version, sizes and checksum of len bytes at buf; copies the header out.
// VMC_OK or VMC_EINVAL (a truncated, damaged or foreign buffer).
int ckpt_validate(const void* buf, size_t len, CkptHeader* out);

}  // namespace vmc_host
