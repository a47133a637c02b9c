// Several-beta kernel instances for FP8 storage.
#include "multi_inst.hpp"

namespace glmrt {

MultiInst multi_pick_fp8(int lpr, int cpl, int nb) {
    return multi_detail::mpick_nb<glmk::DT_FP8>(lpr, cpl, nb);
}

}  // namespace glmrt
