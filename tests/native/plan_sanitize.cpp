// Drives the library's host-side planning code (configuration checks, workspace layout, the
// per-kernel work lists of uneven batches) for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer, without a GPU: pimd_workspace_bytes over batches of 1 to 300
// replicas of uneven N (1 to 5000), both precisions, d = 1..3, two species, every flag
// combination that changes the plan; invalid configurations (which must be refused); and
// pimd_create with a missing or misaligned workspace (refused before any device call).
// Prints "ok" and the number of plans on success.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/pimd.h"

static int fails = 0;
#define CHECK(c, what)                                        \
  do {                                                        \
    if (!(c)) {                                               \
      std::fprintf(stderr, "FAILED %s\n", what);              \
      ++fails;                                                \
    }                                                         \
  } while (0)

static pimd_replica replica(int n, int n2, double xi, double amp) {
  pimd_replica q;
  std::memset(&q, 0, sizeof(q));
  q.n = n; q.n2 = n2; q.beta = 3.0; q.hbar = 1.0; q.mass = 1.0; q.omega = 1.0; q.xi = xi;
  q.pair_amp = amp; q.pair_width = 0.5; q.dt = 0.01; q.nhc_q = 0.0; q.bead_mass = 0.0;
  return q;
}

static pimd_config config(const std::vector<pimd_replica>& reps, int p, int dim, int precision, int flags,
                          int rec_wg) {
  pimd_config c;
  std::memset(&c, 0, sizeof(c));
  c.n_replicas = (int32_t)reps.size(); c.p = p; c.dim = dim; c.precision = precision; c.nhc_len = 4;
  c.sy_order = 3; c.density_bins = 32; c.trace_capacity = 8; c.recursion_workgroups = rec_wg;
  c.flags = flags; c.density_rmax = 4.0; c.replicas = reps.data();
  return c;
}

int main() {
  CHECK(pimd_abi_version() == PIMD_ABI_VERSION, "abi version");
  int plans = 0;
  uint64_t state = 0x9E3779B97F4A7C15ull;
  auto rnd = [&](int lo, int hi) {
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return lo + (int)(state % (uint64_t)(hi - lo + 1));
  };
  const int counts[] = {1, 2, 7, 64, 128, 300};
  const int flag_sets[] = {0, PIMD_FLAG_PAIR_ORDERED, PIMD_FLAG_NO_PERSISTENT, PIMD_FLAG_LONGEST_FIRST,
                           PIMD_FLAG_PAIR_SPLIT_1, 2 * PIMD_FLAG_PAIR_SPLIT_1, 3 * PIMD_FLAG_PAIR_SPLIT_1,
                           PIMD_FLAG_RECURSION_WIDE, PIMD_FLAG_GRAPH};
  for (int R : counts)
    for (int dim = 1; dim <= 3; ++dim)
      for (int prec = 0; prec <= 1; ++prec)
        for (int fl : flag_sets) {
          std::vector<pimd_replica> reps;
          for (int r = 0; r < R; ++r) {
            const int n = R <= 2 ? (r == 0 ? 1 : 5000) : rnd(1, R >= 128 ? 700 : 2000);
            const int n2 = (r % 3 == 2 && n >= 2) ? n / 3 : 0;
            reps.push_back(replica(n, n2, 0.2 * (1 + r % 5), r % 4 == 1 ? 0.0 : 0.5));
          }
          for (int rec_wg : {0, 1, 5}) {
            for (int p : {2, 12, 32}) {
              pimd_config c = config(reps, p, dim, prec, fl, rec_wg);
              size_t bytes = 0;
              CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_OK, "workspace_bytes");
              CHECK(bytes > 0, "workspace size");
              ++plans;
              pimd_ctx* ctx = nullptr;
              CHECK(pimd_create(&c, nullptr, bytes, nullptr, &ctx) == PIMD_ERR_WORKSPACE && ctx == nullptr,
                    "create refuses a missing workspace");
              CHECK(pimd_create(&c, reinterpret_cast<void*>(uintptr_t(4096 + 8)), bytes, nullptr, &ctx) ==
                        PIMD_ERR_WORKSPACE,
                    "create refuses a misaligned workspace");
              CHECK(pimd_create(&c, reinterpret_cast<void*>(uintptr_t(4096)), bytes - 1, nullptr, &ctx) ==
                        PIMD_ERR_WORKSPACE,
                    "create refuses a short workspace");
            }
          }
        }
  // invalid configurations
  std::vector<pimd_replica> one = {replica(10, 0, 1.0, 0.5)};
  size_t bytes = 0;
  pimd_config c = config(one, 32, 2, 1, 0, 0);
  CHECK(pimd_workspace_bytes(nullptr, &bytes) == PIMD_ERR_INVALID, "NULL config");
  CHECK(pimd_workspace_bytes(&c, nullptr) == PIMD_ERR_INVALID, "NULL bytes");
  c.p = 1;
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "p = 1");
  c = config(one, 32, 4, 1, 0, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "dim = 4");
  c = config(one, 32, 2, 1, 1 << 20, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "unknown flag");
  c = config(one, 32, 2, 7, 0, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "unknown precision");
  std::vector<pimd_replica> badrep = {replica(0, 0, 1.0, 0.5)};
  c = config(badrep, 32, 2, 1, 0, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "n = 0");
  badrep = {replica(10, 10, 1.0, 0.5)};
  c = config(badrep, 32, 2, 1, 0, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "n2 = n");
  badrep = {replica(10, 0, -0.5, 0.5)};
  c = config(badrep, 32, 2, 1, 0, 0);
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "xi < 0");
  c = config(one, 32, 2, 1, 0, 0);
  c.n_replicas = 0;
  CHECK(pimd_workspace_bytes(&c, &bytes) == PIMD_ERR_INVALID, "no replicas");
  CHECK(pimd_last_error() != nullptr && std::strlen(pimd_last_error()) > 0, "last error message");
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("ok %d\n", plans);
  return 0;
}
