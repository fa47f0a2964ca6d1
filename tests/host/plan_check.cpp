// Host-side checks of the build planning arithmetic (no GPU, no HIP):
// compiled with g++ by tests/test_host_plan.py.
#include <stdio.h>
#include <stdlib.h>

#include "build_plan.hpp"

using namespace compass;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);           \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main() {
  const int64_t tile = 8192;
  // fused scan chunks: a multiple of the tile, never above INT32_MAX rows
  for (int64_t n : {(int64_t)1, (int64_t)8191, (int64_t)8193,
                    (int64_t)36000000, (int64_t)1 << 31, ((int64_t)1 << 40) + 17,
                    ((int64_t)1 << 47) - 1}) {
    for (int64_t c : {(int64_t)1, (int64_t)3, (int64_t)146, (int64_t)4096}) {
      const int64_t r = fused_rows_per_chunk(n, c, tile);
      CHECK(r % tile == 0);
      CHECK(r >= tile);
      CHECK(r <= (int64_t)INT32_MAX);
      const int64_t chunks = (n + r - 1) / r;
      CHECK(chunks >= 1);
      CHECK(chunks * r >= n);
      // as many chunks as asked for whenever the int32 bound allows it
      if ((n + c - 1) / c <= (int64_t)INT32_MAX / tile * tile - tile)
        CHECK(chunks <= c);
    }
  }
  CHECK(fused_rows_per_chunk((int64_t)1 << 40, 1, tile) == (int64_t)INT32_MAX / tile * tile);

  // LDS guard with a forced budget: the kernel that once faulted needed
  // 128 KiB of dynamic plus 32776 bytes of static LDS, 8 bytes above the
  // 160 KiB a workgroup may allocate
  CHECK(!lds_fits(131072, 32776, 163840));
  CHECK(lds_fits(131072, 32768, 163840));
  CHECK(lds_fits(0, 0, 0));
  CHECK(!lds_fits(65536, 8, 65536));

  // two-phase plan of the 1B-row scan: 6 sketches, d = 11, w = 65536
  {
    const size_t budget = ((size_t)17) << 29;
    const TwoPhasePlan p =
        plan_two_phase(1000000000, 6, 11, 65536, 256, budget, 0, 4096, 48);
    CHECK(p.ok);
    CHECK(p.ranges == 1);
    CHECK(p.total_bytes <= budget);
    CHECK(p.cap >= 2 * p.batch);
    CHECK(p.batch % 4096 == 0 && p.batch >= 4096);
    CHECK(p.slab_bytes >= (size_t)p.chunks * 66 * 65536 * 4);
    CHECK(p.slab_bytes <= budget / 4 + 256);
    // the flush's workgroups fill whole waves of the 256 CUs well
    const int items = 66 * p.chunks;
    const int waves = (items + 255) / 256;
    CHECK((double)items / (waves * 256) > 0.9);
    CHECK(p.surv_bytes >= (size_t)p.cap * 6 * 8);
    printf("large: cap %lld batch %lld chunks %d total %zu\n", (long long)p.cap,
           (long long)p.batch, p.chunks, p.total_bytes);
  }
  // a table whose worst case fits: one batch, no flush before the end
  {
    const TwoPhasePlan p =
        plan_two_phase(2500000, 1, 7, 8192, 256, ((size_t)17) << 29, 0, 4096, 48);
    CHECK(p.ok);
    CHECK(p.batch == p.cap);
    CHECK(p.cap >= 2500000);
  }
  // a cap override gives batches of half the cap
  {
    const TwoPhasePlan p =
        plan_two_phase(3000000, 2, 5, 65536, 256, ((size_t)17) << 29, 100000, 4096, 48);
    CHECK(p.ok);
    CHECK(p.cap == 98304);
    CHECK(p.batch == 49152);
  }
  // a cap below two tiles cannot hold one batch
  {
    const TwoPhasePlan p =
        plan_two_phase(3000000, 2, 5, 65536, 256, ((size_t)17) << 29, 4096, 4096, 48);
    CHECK(!p.ok);
  }
  // a fixed region too small for one slab row, and one just big enough
  {
    const TwoPhasePlan p = plan_two_phase(1000000, 6, 11, 65536, 256,
                                          (size_t)16 << 20, 0, 4096, 48);
    CHECK(!p.ok);
    const TwoPhasePlan q = plan_two_phase(1000000, 1, 1, 65536, 256,
                                          (size_t)16 << 20, 0, 4096, 48);
    CHECK(q.ok);
    CHECK(q.total_bytes <= ((size_t)16 << 20));
  }
  printf(fails ? "FAILED %d\n" : "ALL OK\n", fails);
  return fails ? 1 : 0;
}
