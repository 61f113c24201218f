// Collision and adjoint pipelines, double, padded grid P = 128: every compiled tile shape.
#include "qb_pipelines.hpp"

template bool collision_pipeline<double, 128, 32>(qb_plan_s*, const double*, double*, int, int, hipStream_t);
template bool collision_vjp_pipeline<double, 128, 32>(qb_plan_s*, const double*, const double*, double*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<double, 128, 16>(qb_plan_s*, const double*, double*, int, int, hipStream_t);
template bool collision_vjp_pipeline<double, 128, 16>(qb_plan_s*, const double*, const double*, double*, int, int,
                                                   hipStream_t);
