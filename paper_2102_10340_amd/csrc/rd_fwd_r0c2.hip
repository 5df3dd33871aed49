// Forward kernel instances: recording mode 0, 2 column(s) per lane (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r0c2, 0, 2, kMaxDepthCpl2)
}  // namespace rd
