// Continuous-batching server (internal).
#pragma once

#include "core.hpp"

namespace tnc {

struct Server;
std::shared_ptr<Server> make_server(Ctx& ctx, int max_inflight, int queue_cap);

}  // namespace tnc
