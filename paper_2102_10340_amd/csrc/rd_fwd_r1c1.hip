// Forward kernel instances: recording mode 1, 1 column(s) per lane (rd_fwd_kernel.h).
#include "rd_fwd_kernel.h"

namespace rd {
RD_STREAM_TABLE(stream_fn_r1c1, 1, 1, kMaxDepthCpl1)
}  // namespace rd
