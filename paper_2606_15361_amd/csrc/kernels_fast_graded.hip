// Instances of the specialised LDS row-group kernel for the graded tree mode.
#include "group_fast.h"

namespace snd {

int launch_group_fast_graded(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nb)
{
    hipStream_t st = (hipStream_t)stream;
    if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U8) return launch_fast_typed<SND_MODE_GRADED, uint8_t, uint8_t>(a, n_out, lds, st, m, nb);
    if (src_dt == SND_DT_U16 && dst_dt == SND_DT_U16) return launch_fast_typed<SND_MODE_GRADED, uint16_t, uint16_t>(a, n_out, lds, st, m, nb);
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
