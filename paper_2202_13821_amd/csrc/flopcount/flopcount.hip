// Host instantiations of the device point functions, compiled to optimised
// LLVM IR by count_flops.py to count the floating-point operations of one
// face point and one volume point (straight-line code after unrolling).
#include "../gks_point.hpp"

using namespace dgk;

#define FACE(T, NF, name)                                                                               \
  extern "C" void name(const Phys* ph, const T* qL, const T (*dqL)[5], const T* qR, const T (*dqR)[5], T* F, \
                       T* Ft, int* bad) {                                                               \
    face_flux_local<T, NF>(*ph, qL, dqL, qR, dqR, F, Ft, *bad);                                         \
  }
#define VOL(T, NF, name)                                                                                       \
  extern "C" void name(const Phys* ph, const T* q, const T (*dq)[5], T (*F)[5], T (*Ft)[5], int* bad) { \
    volume_flux<T, NF>(*ph, q, dq, F, Ft, *bad);                                                               \
  }
FACE(float, true, fc_face_f32_s1)
FACE(float, false, fc_face_f32_s2)
FACE(double, true, fc_face_f64_s1)
FACE(double, false, fc_face_f64_s2)
VOL(float, true, fc_vol_f32_s1)
VOL(float, false, fc_vol_f32_s2)
VOL(double, true, fc_vol_f64_s1)
VOL(double, false, fc_vol_f64_s2)

// Pieces of the adjoint: one side and the finish of the face flux (forward,
// recomputed by the adjoint), and the reverses of the side, the finish and
// the volume flux.
#include "../gks_point_adj.hpp"

#define SIDE(T, name)                                                                                  \
  extern "C" void name(const Phys* ph, const T* q, const T (*dq)[5], FaceAcc<T>* acc, int* bad) {       \
    face_side(*ph, q, dq, *acc, *bad, T(1));                                                           \
  }
#define SIDE_VJP(T, name)                                                                                        \
  extern "C" void name(const Phys* ph, const T* q, const T (*dq)[5], const FaceAcc<T>* accb, T* qb, T (*dqb)[5]) { \
    face_side_vjp(*ph, q, dq, *accb, qb, dqb, T(1));                                                             \
  }
#define FINISH_VJP(T, NF, name)                                                                                \
  extern "C" void name(const Phys* ph, const FaceAcc<T>* acc, const T* Fb, const T* Ftb, FaceAcc<T>* accb,     \
                       double* mub) {                                                                         \
    face_finish_vjp<T, NF>(*ph, *acc, Fb, Ftb, *accb, *mub);                                                  \
  }
#define VOL_VJP(T, NF, name)                                                                                   \
  extern "C" void name(const Phys* ph, const T* q, const T (*dq)[5], const T (*Fb)[5], const T (*Ftb)[5], T* qb, \
                       T (*dqb)[5], double* mub) {                                                            \
    volume_flux_vjp<T, NF>(*ph, q, dq, Fb, Ftb, qb, dqb, *mub);                                               \
  }
SIDE(float, fc_side_f32)
SIDE(double, fc_side_f64)
SIDE_VJP(float, fc_sidevjp_f32)
SIDE_VJP(double, fc_sidevjp_f64)
FINISH_VJP(float, true, fc_finvjp_f32_s1)
FINISH_VJP(float, false, fc_finvjp_f32_s2)
FINISH_VJP(double, true, fc_finvjp_f64_s1)
FINISH_VJP(double, false, fc_finvjp_f64_s2)
VOL_VJP(float, true, fc_volvjp_f32_s1)
VOL_VJP(float, false, fc_volvjp_f32_s2)
VOL_VJP(double, true, fc_volvjp_f64_s1)
VOL_VJP(double, false, fc_volvjp_f64_s2)
