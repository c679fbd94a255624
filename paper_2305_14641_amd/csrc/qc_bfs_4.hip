// Multi-source BFS instantiations for a batch width of 4 sources.
#include "qc_bfs.h"

namespace qc {
template hipError_t launch_bfs_bw<4>(int, int, int, const GraphDev *, const BfsJob *, int,
                                         hipStream_t);
}  // namespace qc
