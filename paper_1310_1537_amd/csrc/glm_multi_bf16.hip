// Several-beta kernel instances for BF16 storage.
#include "multi_inst.hpp"

namespace glmrt {

MultiInst multi_pick_bf16(int lpr, int cpl, int nb) {
    return multi_detail::mpick_nb<glmk::DT_BF16>(lpr, cpl, nb);
}

}  // namespace glmrt
