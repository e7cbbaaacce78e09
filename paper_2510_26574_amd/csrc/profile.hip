// Event-pair pool behind the per-kernel timing hooks (see profile.hpp).
#include "profile.hpp"

#include <vector>

#include "common.hpp"

namespace prof {
namespace {
constexpr int POOL = 8192;
bool g_on = false;
struct Pair {
  hipEvent_t a, b;
  int kind;
};
std::vector<Pair> g_pool;
int g_used = 0;
int g_open = -1;
bool g_overflow = false;
}  // namespace

bool enabled() { return g_on; }

void begin(int kind, hipStream_t st) {
  if (!g_on) return;
  if (g_used >= (int)g_pool.size()) {
    g_overflow = true;
    g_open = -1;
    return;
  }
  g_open = g_used++;
  g_pool[g_open].kind = kind;
  (void)hipEventRecord(g_pool[g_open].a, st);
}

void end(int kind, hipStream_t st) {
  if (!g_on || g_open < 0) return;
  (void)kind;
  (void)hipEventRecord(g_pool[g_open].b, st);
  g_open = -1;
}
}  // namespace prof

extern "C" int rpc_profile_enable(int on) {
  if (on && prof::g_pool.empty()) {
    prof::g_pool.resize(prof::POOL);
    for (auto& p : prof::g_pool) {
      if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return RPC_EHIP;
    }
  }
  prof::g_on = on != 0;
  return RPC_OK;
}

extern "C" int rpc_profile_reset(void) {
  prof::g_used = 0;
  prof::g_open = -1;
  prof::g_overflow = false;
  return RPC_OK;
}

extern "C" int rpc_profile_read(int32_t kind, double* total_ms, int64_t* launches) {
  if (!total_ms || !launches || kind < 0 || kind >= prof::NKIND) return RPC_EINVAL;
  double t = 0.0;
  int64_t n = 0;
  for (int i = 0; i < prof::g_used; ++i) {
    if (prof::g_pool[i].kind != kind) continue;
    if (hipEventSynchronize(prof::g_pool[i].b) != hipSuccess) return RPC_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, prof::g_pool[i].a, prof::g_pool[i].b) != hipSuccess) return RPC_EHIP;
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return prof::g_overflow ? RPC_EWORKSPACE : RPC_OK;
}
