// instantiate.hip -- explicit instantiation of the launch code for one
// configuration, selected at compile time with -DDGK_T=float|double
// -DDGK_K=<degree> -DDGK_NQ=<points per axis> (one object file each, so the
// configurations compile in parallel).
#include "launch.hpp"

#if !defined(DGK_T) || !defined(DGK_K) || !defined(DGK_NQ)
#error "instantiate.hip needs DGK_T, DGK_K and DGK_NQ"
#endif

namespace dgrt {
template int run_step<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, double*, double, int, double*, int);
template int run_residual<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, const double*, double, double*, double*);
template int run_adjoint<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, const double*, int, double, int, const double*,
                                               double*, double*);
}  // namespace dgrt
