// Collision and adjoint pipelines, float, padded grid P = 64: every compiled tile shape.
#include "qb_pipelines.hpp"

template bool collision_pipeline<float, 64, 32>(qb_plan_s*, const float*, float*, int, int, hipStream_t);
template bool collision_vjp_pipeline<float, 64, 32>(qb_plan_s*, const float*, const float*, float*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<float, 64, 16>(qb_plan_s*, const float*, float*, int, int, hipStream_t);
template bool collision_vjp_pipeline<float, 64, 16>(qb_plan_s*, const float*, const float*, float*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<float, 64, 8>(qb_plan_s*, const float*, float*, int, int, hipStream_t);
template bool collision_vjp_pipeline<float, 64, 8>(qb_plan_s*, const float*, const float*, float*, int, int,
                                                  hipStream_t);
