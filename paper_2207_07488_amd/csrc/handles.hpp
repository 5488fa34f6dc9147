// Definitions of the opaque ABI handles (shared by api.cpp and serve.cpp).
#pragma once
#include <memory>

#include "internal.hpp"

struct sn_network_s {
  std::shared_ptr<spnet::Network> p;
};
struct sn_system_s {
  std::shared_ptr<spnet::System> p;
};
struct sn_precond_s {
  std::shared_ptr<spnet::Precond> p;
};

namespace spnet {
// Runs fn, turning exceptions into a status and the thread's error message.
sn_status guarded_call(void (*fn)(void *), void *ctx);
template <typename Fn>
sn_status guarded(Fn fn) {
  return guarded_call([](void *c) { (*static_cast<Fn *>(c))(); }, &fn);
}
}  // namespace spnet
