// instantiate.hip -- explicit instantiation of the launch code for one
// configuration, selected at compile time with -DDGK_T=float|double
// -DDGK_K=<degree> -DDGK_NQ=<points per axis> (one object file each, so the
// configurations compile in parallel), and -DDGK_PART=1 (the step and the
// operator evaluation, with the stage launches and the face passes), 2 (the
// adjoint, with its face passes), 3 (the adjoint's volume passes) or 4 (the
// forward volume passes).
//
// The parts are separate objects so that each can be compiled with its own
// code-generation options.  Each part calls the launches of the others
// through the declarations marked extern below, so every kernel is compiled
// exactly once.
#include "launch.hpp"

#if !defined(DGK_T) || !defined(DGK_K) || !defined(DGK_NQ) || !defined(DGK_PART)
#error "instantiate.hip needs DGK_T, DGK_K, DGK_NQ and DGK_PART"
#endif

namespace dgrt {
#if DGK_PART == 1
extern template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 0>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&,
                                                                const Geo&, const Phys&);
extern template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&,
                                                                const Geo&, const Phys&);
extern template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 2>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&,
                                                                const Geo&, const Phys&);
template int launch_stage<DGK_T, DGK_K, DGK_NQ, 0>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&, const Geo&,
                                                   const Phys&);
template int launch_stage<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&, const Geo&,
                                                   const Phys&);
template int run_step<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, double*, double, int, double*, int);
template int run_residual<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, const double*, double, double*, double*);
#elif DGK_PART == 2
extern template int launch_stage<DGK_T, DGK_K, DGK_NQ, 0>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&,
                                                          const Geo&, const Phys&);
extern template int launch_stage<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&,
                                                          const Geo&, const Phys&);
extern template int launch_adj_volume<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const AdjIn<1>&, double*,
                                                               const Geo&, const Phys&);
extern template int launch_adj_volume<DGK_T, DGK_K, DGK_NQ, 2>(dg_hgks_ctx*, const DGK_T*, const AdjIn<2>&, double*,
                                                               const Geo&, const Phys&);
template int run_adjoint<DGK_T, DGK_K, DGK_NQ>(dg_hgks_ctx*, const double*, int, double, int, const double*,
                                               double*, double*);
#elif DGK_PART == 3
template int launch_adj_volume<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const AdjIn<1>&, double*,
                                                        const Geo&, const Phys&);
template int launch_adj_volume<DGK_T, DGK_K, DGK_NQ, 2>(dg_hgks_ctx*, const DGK_T*, const AdjIn<2>&, double*,
                                                        const Geo&, const Phys&);
#elif DGK_PART == 4
template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 0>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&, const Geo&,
                                                         const Phys&);
template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 1>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&, const Geo&,
                                                         const Phys&);
template int launch_volume_pass<DGK_T, DGK_K, DGK_NQ, 2>(dg_hgks_ctx*, const DGK_T*, const VolOut<DGK_T>&, const Geo&,
                                                         const Phys&);
#else
#error "DGK_PART is 1 (forward), 2 (adjoint), 3 (adjoint volume passes) or 4 (forward volume passes)"
#endif
}  // namespace dgrt
