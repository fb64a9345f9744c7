// Runtime dispatch from (N, M, dtype, mode) to the compiled kernel instances.
#include <hip/hip_runtime.h>

#include "bbwadg_internal.hpp"

namespace bbw {

#define BBW_DECL(NN)                                                                                  \
  int launch_stage_n##NN(int M, bool update, bool f64, const void* args, void* stream);             \
  int launch_l2norm_n##NN(bool f64, const void* q, int64_t K, const double* J, const double* mass, \
                          double* partial, int nblocks, void* stream);
BBW_DECL(1) BBW_DECL(2) BBW_DECL(3) BBW_DECL(4) BBW_DECL(5) BBW_DECL(6) BBW_DECL(7) BBW_DECL(8) BBW_DECL(9)
#undef BBW_DECL

static int stage(int N, int M, bool update, bool f64, const void* args, void* stream) {
  switch (N) {
    case 1: return launch_stage_n1(M, update, f64, args, stream);
    case 2: return launch_stage_n2(M, update, f64, args, stream);
    case 3: return launch_stage_n3(M, update, f64, args, stream);
    case 4: return launch_stage_n4(M, update, f64, args, stream);
    case 5: return launch_stage_n5(M, update, f64, args, stream);
    case 6: return launch_stage_n6(M, update, f64, args, stream);
    case 7: return launch_stage_n7(M, update, f64, args, stream);
    case 8: return launch_stage_n8(M, update, f64, args, stream);
    case 9: return launch_stage_n9(M, update, f64, args, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_stage_f64(int N, int M, bool update, const StageArgs<double>& a, void* stream) {
  return stage(N, M, update, true, &a, stream);
}
int launch_stage_f32(int N, int M, bool update, const StageArgs<float>& a, void* stream) {
  return stage(N, M, update, false, &a, stream);
}

int launch_l2norm(int N, int dtype, const void* q, int64_t K, const double* J, const double* mass, double* partial,
                  int nblocks, void* stream) {
  const bool f64 = dtype == 0;
  switch (N) {
    case 1: return launch_l2norm_n1(f64, q, K, J, mass, partial, nblocks, stream);
    case 2: return launch_l2norm_n2(f64, q, K, J, mass, partial, nblocks, stream);
    case 3: return launch_l2norm_n3(f64, q, K, J, mass, partial, nblocks, stream);
    case 4: return launch_l2norm_n4(f64, q, K, J, mass, partial, nblocks, stream);
    case 5: return launch_l2norm_n5(f64, q, K, J, mass, partial, nblocks, stream);
    case 6: return launch_l2norm_n6(f64, q, K, J, mass, partial, nblocks, stream);
    case 7: return launch_l2norm_n7(f64, q, K, J, mass, partial, nblocks, stream);
    case 8: return launch_l2norm_n8(f64, q, K, J, mass, partial, nblocks, stream);
    case 9: return launch_l2norm_n9(f64, q, K, J, mass, partial, nblocks, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace bbw
