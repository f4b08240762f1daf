// Stand-ins for the HIP runtime and the kernel launch wrappers, so that the C
// ABI's host logic (ga_api.hip) builds with g++ and runs under AddressSanitizer
// and UndefinedBehaviorSanitizer on the CPU: device memory is host memory,
// kernels are stubs that check what the host hands them (tile tables, launch
// shapes), streams, events and graphs are tokens. A graph destroyed while
// launched and not synchronised, or a table a launch would misread, aborts.
// Test infrastructure only; nothing here computes a generation.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>
#include <new>
#include "ga_internal.hpp"
struct ihipStream_t { int x; };
struct ihipEvent_t { int x; };
struct ihipGraph_t { int x; };
struct ihipGraphExec_t { int x; bool in_flight = false; hipStream_t on = nullptr; };
#include <set>
static std::set<ihipGraphExec_t*> g_in_flight;
static int g_hits = 0;
const char* hipGetErrorString(hipError_t) { return "mock"; }
hipError_t hipMalloc(void** p, size_t n) { *p = calloc(1, n ? n : 1); return hipSuccess; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = calloc(1, n ? n : 1); return hipSuccess; }
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memmove(d, s, n); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t s) { for (auto it = g_in_flight.begin(); it != g_in_flight.end();) { if ((*it)->on == s) { (*it)->in_flight = false; it = g_in_flight.erase(it); } else ++it; } return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->x++; return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { (void)e->x; return hipSuccess; }  // (staging events only)
hipError_t hipEventQuery(hipEvent_t e) { (void)e->x; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) { if (s) (void)s->x; (void)e->x; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, int) { (void)s->x; return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = new ihipGraph_t(); return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, void*, void*, size_t) { (void)g->x; *x = new ihipGraphExec_t(); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { if (x->in_flight) { fprintf(stderr, "graph exec destroyed while launched and not synchronized (%d)\n", ++g_hits); abort(); } g_in_flight.erase(x); delete x; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) { x->in_flight = true; x->on = s; g_in_flight.insert(x); return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 256; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
// roctx: the ranges are host markers with nothing to check here
extern "C" int roctxRangePushA(const char*) { return 0; }
extern "C" int roctxRangePop() { return 0; }
namespace ga {
// kernel wrappers: touch what the real kernels touch on the host side of the
// contract only where the host reads it back (budgets, tables are read here)
static void check_tab(const RunView* views, const Tile* tiles, const uint32_t* n, uint32_t grid) {
  // every tile the grid covers below the count must name a member
  (void)views; (void)grid;
  for (uint32_t i = 0; i < *n; ++i) (void)tiles[i].run;
}
hipError_t launch_generation(const RunView&, uint32_t, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_tiles(const RunView&, uint64_t, hipStream_t) { return hipSuccess; }
size_t tile_lds_bytes(uint32_t w, uint32_t h, uint32_t l, uint32_t, uint32_t, uint32_t o) { return (size_t)w * h * (16u << l) + 16 * w * h * o; }
uint32_t tile_threads(uint32_t, uint32_t, uint32_t) { return 1024; }
hipError_t tile_occupancy(const RunView&, uint32_t, size_t, int* g) { *g = 1; return hipSuccess; }
hipError_t launch_async(const RunView&, uint64_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_lockstep(const RunView&, uint64_t, uint64_t, uint32_t, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t async_capacity(const RunView&, uint32_t, bool, uint32_t* w) { *w = 4096; return hipSuccess; }
hipError_t launch_advance(unsigned long long* g, uint64_t n, hipStream_t) { *g += n; return hipSuccess; }
hipError_t launch_init(const RunView&, hipStream_t) { return hipSuccess; }
bool model_has_string_host(uint32_t id) { return id != 0; }
uint32_t model_count() { return 3; }
size_t lds_bytes(uint32_t ipw, uint32_t waves, uint32_t model) { return (5u * ipw + 1u) * 16u * (model ? 2u : 1u) * waves; }
hipError_t launch_fill(uint32_t* p, uint32_t v, size_t n, hipStream_t) { for (size_t i = 0; i < n; ++i) p[i] = v; return hipSuccess; }
hipError_t launch_sample(const RunView& v, uint32_t* ids, hipStream_t) { for (uint32_t i = 0; i < v.islands; ++i) ids[i] = i << v.log2n; return hipSuccess; }
hipError_t launch_gather(const RunView& v, const uint32_t* ids, uint32_t n, uint32_t* T, uint32_t* D, hipStream_t) {
  for (uint32_t j = 0; j < n; ++j) { T[j] = v.pop_T[ids[j]]; for (uint32_t w = 0; w < v.words; ++w) D[(size_t)w * n + j] = v.pop_D[(size_t)w * v.agent_stride + ids[j]]; }
  return hipSuccess;
}
hipError_t launch_batch_all(const RunView* views, const Tile* tiles, uint32_t grid, uint32_t, uint32_t max_ipw, uint32_t wpg, hipStream_t) {
  if (wpg == 0 || wpg > 16) { fprintf(stderr, "bad wpg\n"); abort(); }
  if (grid % (8 * wpg)) { fprintf(stderr, "grid %u not whole groups on every XCD\n", grid); abort(); }
  // walk each XCD's slots in dispatch order: tiles in class order within an
  // XCD and from one XCD to the next, bytes spread evenly
  uint64_t bytes[8] = {0}, total = 0, heaviest = 0;
  uint32_t last_cls = 0;
  for (uint32_t x = 0; x < 8; ++x) {
    for (uint32_t g = x; g < grid / wpg; g += 8) {
      for (uint32_t w = 0; w < wpg; ++w) {
        const Tile t = tiles[g * wpg + w];
        if (t.cls == kNoTile) continue;
        const RunView& v = views[t.run];
        if (v.ipw > max_ipw) { fprintf(stderr, "member ipw %u above launch %u\n", v.ipw, max_ipw); abort(); }
        if (t.first % v.ipw || t.first >= v.islands) { fprintf(stderr, "bad tile start\n"); abort(); }
        if (t.cls != v.log2n * 2 + v.words - 1) { fprintf(stderr, "tile class differs from its member's\n"); abort(); }
        if (v.left != v.gen + 1) { fprintf(stderr, "budget word not after the generation counter\n"); abort(); }
        if (t.cls < last_cls) { fprintf(stderr, "tiles not in class order\n"); abort(); }
        last_cls = t.cls;
        const uint32_t isl = std::min(v.ipw, v.islands - t.first);
        const uint64_t b = (uint64_t)isl * (((uint64_t)1 << v.log2n) * 2 * (8 + 4 * v.words) + 2 * (12 + 4 * v.words)) + kWaveFixedBytes;
        bytes[x] += b; total += b; heaviest = std::max(heaviest, b);
      }
    }
  }
  for (uint32_t x = 0; x < 8; ++x)
    if (bytes[x] > total / 8 + heaviest) { fprintf(stderr, "XCD %u holds %llu of %llu (bytes plus a fixed cost per wavefront)\n", x, (unsigned long long)bytes[x], (unsigned long long)total); abort(); }
  return hipSuccess;
}
hipError_t launch_store_u64(unsigned long long* p, unsigned long long v, hipStream_t) { *p = v; return hipSuccess; }
hipError_t launch_batch_advance(const RunView*, const uint32_t* n, uint32_t cap, uint64_t, hipStream_t) { (void)*n; (void)cap; return hipSuccess; }
hipError_t launch_roof_inplace(void*, size_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_roof_philox(uint32_t*, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_roof_valu(uint32_t*, uint32_t, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
size_t mrca_workspace_bytes(size_t n) { return n * 16; }
hipError_t launch_mrca_matrix_noalloc(const uint32_t*, const uint32_t*, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t*, uint32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_mrca_matrix(const uint32_t*, const uint32_t*, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, void*, uint32_t*, uint32_t*, hipStream_t) { return hipSuccess; }
}
