// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host code
// (argument validation and workspace sizing of the C ABI in include/wsr.h): every entry point
// with the invalid arguments it must reject before anything reaches the device, and the
// workspace sizes of valid layouts (short, long, empty and maximal segments).  Runs on a machine
// without a GPU: no call below launches a kernel.  Exits 1 when a call returns another code than
// the expected one; the sanitizers abort on any memory or undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/wsr.h"

static int failures = 0;
static void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "FAIL: %s returned %d, expected %d\n", what, got, want);
    ++failures;
  }
}

int main() {
  std::printf("version %d\n", wsr_version());
  for (int s = -10; s <= 2; ++s)
    if (!wsr_status_string(s)) {
      std::fprintf(stderr, "FAIL: no status string for %d\n", s);
      ++failures;
    }
  // workspace sizes of valid layouts (host arithmetic only)
  size_t bytes = 0;
  const std::vector<std::vector<int64_t>> good = {
      {0},
      {0, 0, 1, 2, 4096, 4097, 8192, 8193},
      {0, 3072, 6144, 20000, 20000, 120000},
      {0, (int64_t)1 << 24},
      {0, (int64_t)1 << 27},
  };
  for (const auto& off : good) {
    expect(wsr_workspace_bytes(off.data(), (int64_t)off.size() - 1, &bytes), WSR_OK, "workspace_bytes(valid)");
    int64_t longest = 0;
    for (size_t i = 0; i + 1 < off.size(); ++i) longest = off[i + 1] - off[i] > longest ? off[i + 1] - off[i] : longest;
    if (longest > 8192 && bytes == 0) {
      std::fprintf(stderr, "FAIL: no workspace for a long segment\n");
      ++failures;
    }
  }
  // invalid layouts
  const int64_t decreasing[] = {0, 10, 5};
  const int64_t nonzero_first[] = {3, 10};
  const int64_t too_long[] = {0, ((int64_t)1 << 27) + 1};
  expect(wsr_workspace_bytes(decreasing, 2, &bytes), WSR_ERR_INVALID, "workspace_bytes(decreasing)");
  expect(wsr_workspace_bytes(nonzero_first, 1, &bytes), WSR_ERR_INVALID, "workspace_bytes(offsets[0] != 0)");
  expect(wsr_workspace_bytes(too_long, 1, &bytes), WSR_ERR_UNSUPPORTED, "workspace_bytes(too long)");
  expect(wsr_workspace_bytes(nullptr, 1, &bytes), WSR_ERR_INVALID, "workspace_bytes(null offsets)");
  expect(wsr_workspace_bytes(decreasing, -1, &bytes), WSR_ERR_INVALID, "workspace_bytes(n_seg < 0)");
  // forward / backward / l1 / stats: rejected before any launch
  float buf[16] = {0};
  int32_t perm[16] = {0};
  uint32_t mask[2] = {0};
  const int64_t off16[] = {0, 16};
  char ws[64];
  expect(wsr_prox_forward(nullptr, buf, off16, 1, 0.1f, nullptr, nullptr, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "forward(null w)");
  expect(wsr_prox_forward(buf, buf, off16, 1, -1.0f, nullptr, nullptr, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "forward(lambda < 0)");
  expect(wsr_prox_forward(buf, buf, off16, 1, 0.0f / 0.0f, nullptr, nullptr, ws, sizeof ws, nullptr),
         WSR_ERR_INVALID, "forward(lambda NaN)");
  expect(wsr_prox_forward(buf, buf, decreasing, 2, 0.1f, nullptr, nullptr, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "forward(bad offsets)");
  expect(wsr_prox_forward(buf, buf, off16, 1, 0.1f, perm, nullptr, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "forward(perm without mask)");
  expect(wsr_prox_forward(buf, buf, too_long, 1, 0.1f, nullptr, nullptr, ws, sizeof ws, nullptr),
         WSR_ERR_UNSUPPORTED, "forward(too long)");
  const int64_t long_off[] = {0, 100000};
  expect(wsr_prox_forward(buf, buf, long_off, 1, 0.1f, nullptr, nullptr, ws, sizeof ws, nullptr),
         WSR_ERR_WORKSPACE, "forward(workspace too small)");
  expect(wsr_prox_forward_noalloc(buf, buf, too_long, 1, 0.1f, nullptr, nullptr, nullptr), WSR_ERR_UNSUPPORTED,
         "forward_noalloc(too long)");
  expect(wsr_prox_l1_forward(buf, buf, off16, 1, 0.1f, -1.0f, 0.5f, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "l1_forward(beta < 0)");
  expect(wsr_prox_l1_forward(buf, buf, off16, 1, 0.1f, 0.1f, 1.5f, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "l1_forward(rho > 1)");
  expect(wsr_prox_backward(buf, buf, off16, 1, perm, mask, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "backward(grad_w aliases grad_out)");
  expect(wsr_prox_backward(buf, buf + 8, off16, 1, nullptr, mask, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "backward(null perm)");
  expect(wsr_segment_stats(buf, decreasing, 2, nullptr, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "segment_stats(null stats)");
  // plans: invalid layouts and null handles
  wsr_plan* plan = nullptr;
  expect(wsr_plan_create(decreasing, 2, 0, &plan), WSR_ERR_INVALID, "plan_create(bad offsets)");
  expect(wsr_plan_create(off16, 1, 0, nullptr), WSR_ERR_INVALID, "plan_create(null out)");
  expect(wsr_plan_destroy(nullptr), WSR_ERR_INVALID, "plan_destroy(null)");
  expect(wsr_plan_workspace_bytes(nullptr, &bytes), WSR_ERR_INVALID, "plan_workspace_bytes(null)");
  int32_t rounds[4] = {0};
  expect(wsr_plan_merge_rounds(nullptr, rounds), WSR_ERR_INVALID, "plan_merge_rounds(null)");
  expect(wsr_plan_set_merge_rounds(nullptr, rounds), WSR_ERR_INVALID, "plan_set_merge_rounds(null)");
  expect(wsr_plan_sort_routes(nullptr, rounds), WSR_ERR_INVALID, "plan_sort_routes(null)");
  expect(wsr_plan_set_sort_routes(nullptr, rounds), WSR_ERR_INVALID, "plan_set_sort_routes(null)");
  uint32_t flags = 0;
  expect(wsr_read_status(nullptr, &flags, 0, nullptr), WSR_ERR_INVALID, "read_status(null)");
  expect(wsr_prox_forward_batched(nullptr, buf, buf, nullptr, 0.1f, nullptr, nullptr, ws, sizeof ws, nullptr),
         WSR_ERR_INVALID, "forward_batched(null plan)");
  expect(wsr_prox_backward_batched(nullptr, buf, buf + 8, perm, mask, ws, sizeof ws, nullptr), WSR_ERR_INVALID,
         "backward_batched(null plan)");
  // tracing bookkeeping (host only while nothing is recorded)
  expect(wsr_trace_enable(0), WSR_OK, "trace_enable(0)");
  int n = -1;
  expect(wsr_trace_collect(0, nullptr, nullptr, nullptr, &n), WSR_OK, "trace_collect(empty)");
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("host sanitizer driver: ok\n");
  return 0;
}
