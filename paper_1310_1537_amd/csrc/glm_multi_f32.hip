// Several-beta kernel instances for F32 storage.
#include "multi_inst.hpp"

namespace glmrt {

MultiInst multi_pick_f32(int lpr, int cpl, int nb) {
    return multi_detail::mpick_nb<glmk::DT_F32>(lpr, cpl, nb);
}

}  // namespace glmrt
