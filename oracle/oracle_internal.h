/* TEST INFRASTRUCTURE ONLY -- internal declarations of the CPU oracle. */
#ifndef PAMO_ORACLE_INTERNAL_H
#define PAMO_ORACLE_INTERNAL_H
#include <stdint.h>

/* exact signs (-1, 0, +1) */
int o_orient2d(const double *a, const double *b, const double *c);
int o_orient3d(const double *a, const double *b, const double *c, const double *d);

/* self-intersection predicate between two mesh triangles given by their corner
 * positions and vertex ids (returns 1 if the pair is a self-intersection) */
int o_tri_pair(const double *const P[3], const int32_t ip[3],
               const double *const Q[3], const int32_t iq[3]);

/* exact: is the triangle with these corners collinear (zero area)? */
int o_degenerate(const double *a, const double *b, const double *c);

#endif
