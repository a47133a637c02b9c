// Several-beta kernel instances for F64 storage.
#include "multi_inst.hpp"

namespace glmrt {

MultiInst multi_pick_f64(int lpr, int cpl, int nb) {
    return multi_detail::mpick_nb<glmk::DT_F64>(lpr, cpl, nb);
}

}  // namespace glmrt
