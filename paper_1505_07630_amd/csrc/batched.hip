// Batched solves of many independent systems (placeholder until the
// persistent kernel lands).
#include "handles.hpp"

struct fvpcg_batch {
    int nsys = 0;
    int ncells = 0;
    int nfaces = 0;
};

namespace fvpcg {

int batch_create(int32_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*, const double*,
                 const double*, const double*, uint32_t, hipStream_t, fvpcg_batch**) {
    return set_error(FVPCG_UNSUPPORTED, "batched solver not built");
}
int batch_destroy(fvpcg_batch* bt) {
    delete bt;
    return FVPCG_OK;
}
int batch_total_cells(const fvpcg_batch* bt) { return bt->ncells; }
int batch_total_faces(const fvpcg_batch* bt) { return bt->nfaces; }
int batch_nsys(const fvpcg_batch* bt) { return bt->nsys; }
int solve_batched(const fvpcg_batch*, const double*, double*, double, int, int, int, hipStream_t, fvpcg_stats*) {
    return set_error(FVPCG_UNSUPPORTED, "batched solver not built");
}
int solve_batched_backward(const fvpcg_batch*, const double*, const double*, double*, double*, double*, double*,
                           double, int, int, int, hipStream_t, fvpcg_stats*) {
    return set_error(FVPCG_UNSUPPORTED, "batched solver not built");
}

}  // namespace fvpcg
