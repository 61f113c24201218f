// Collision and adjoint pipelines, double, padded grid P = 64: every compiled tile shape.
#include "qb_pipelines.hpp"

template bool collision_pipeline<double, 64, 32>(qb_plan_s*, const double*, double*, int, int, hipStream_t);
template bool collision_vjp_pipeline<double, 64, 32>(qb_plan_s*, const double*, const double*, double*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<double, 64, 16>(qb_plan_s*, const double*, double*, int, int, hipStream_t);
template bool collision_vjp_pipeline<double, 64, 16>(qb_plan_s*, const double*, const double*, double*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<double, 64, 8>(qb_plan_s*, const double*, double*, int, int, hipStream_t);
template bool collision_vjp_pipeline<double, 64, 8>(qb_plan_s*, const double*, const double*, double*, int, int,
                                                  hipStream_t);
