// Continuous-batching server (internal).
#pragma once

#include <deque>

#include "core.hpp"

namespace tnc {

struct Server;
struct Request;
std::shared_ptr<Server> make_server(Ctx& ctx, int max_inflight, int queue_cap);

// A plan whose batch label's rows are filled from queued row requests.
struct Batcher {
  std::shared_ptr<Plan> plan_ref;
  Plan* plan = nullptr;
  int label = -1;
  int64_t B = 1;                      // rows per batch (the label's extent)
  std::vector<int> leaves;            // leaves carrying the label (outermost)
  std::vector<int64_t> row_elems;     // per listed leaf: numel / B
  int64_t row_total = 0;              // sum of row_elems
  int64_t out_row = 1;                // result elements per row (R / B)
  int64_t work_bytes = 0, need = 0;   // workspace and arena need of one batch
  double flops = 0;                   // planned work of one batch
  // guarded by the server mutex: rows waiting for a batch, whether a batch
  // is running, whether the batcher's token waits in the server queue
  std::deque<std::shared_ptr<Request>> rows;
  bool busy = false;
  bool queued = false;
  ~Batcher();
};

}  // namespace tnc
