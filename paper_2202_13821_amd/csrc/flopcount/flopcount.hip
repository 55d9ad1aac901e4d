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
