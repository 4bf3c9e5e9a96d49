// Instances of the specialised LDS row-group kernel for the float tree mode.
#include "group_fast.h"

namespace snd {

int launch_group_fast_float(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nb)
{
    hipStream_t st = (hipStream_t)stream;
    if (dst_dt != SND_DT_F32) return (int)hipErrorInvalidValue;
    if (src_dt == SND_DT_F32) return launch_fast_typed<SND_MODE_FLOAT, float, float>(a, n_out, lds, st, m, nb);
    if (src_dt == SND_DT_BF16) return launch_fast_typed<SND_MODE_FLOAT, bf16_t, float>(a, n_out, lds, st, m, nb);
    if (src_dt == SND_DT_F16) return launch_fast_typed<SND_MODE_FLOAT, f16_t, float>(a, n_out, lds, st, m, nb);
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
