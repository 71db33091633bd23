// FFT plan table of the solver: one compiled plan per supported axis length,
// every n = 2^a 3^b in [4, 512].
//
// X(G, N, R0, R1, R2, TPC): N = R0 R1 R2 points in up to three Stockham
// stages of radix R0, R1, R2 (1 = no stage); TPC threads cooperate on one
// column, each owning E = N / TPC elements, so TPC must divide N / R for every
// stage radix R.  G is the translation unit (cbs_pass_group.hip built with
// -DCBS_GROUP=G) that compiles the plan's kernels; the groups only spread the
// compile time over parallel jobs.
#pragma once

#define CBS_PLANS(X)                 \
    X(0, 4, 4, 1, 1, 1)              \
    X(0, 6, 6, 1, 1, 1)              \
    X(0, 8, 8, 1, 1, 1)              \
    X(0, 12, 12, 1, 1, 1)            \
    X(0, 16, 4, 4, 1, 4)             \
    X(0, 24, 4, 6, 1, 2)             \
    X(0, 32, 4, 8, 1, 4)             \
    X(0, 48, 4, 12, 1, 4)            \
    X(1, 64, 8, 8, 1, 8)             \
    X(1, 96, 4, 4, 6, 8)             \
    X(2, 128, 8, 16, 1, 8)           \
    X(2, 192, 4, 4, 12, 16)          \
    X(3, 256, 16, 16, 1, 16)         \
    X(4, 512, 8, 8, 8, 64)           \
    X(5, 9, 9, 1, 1, 1)              \
    X(5, 18, 3, 6, 1, 3)             \
    X(5, 27, 3, 9, 1, 3)             \
    X(5, 36, 6, 6, 1, 6)             \
    X(5, 54, 3, 3, 6, 9)             \
    X(5, 72, 6, 12, 1, 6)            \
    X(5, 81, 9, 9, 1, 9)             \
    X(6, 108, 6, 6, 3, 18)           \
    X(6, 144, 12, 12, 1, 12)         \
    X(6, 162, 2, 9, 9, 9)            \
    X(7, 216, 12, 3, 6, 18)          \
    X(7, 243, 3, 9, 9, 27)           \
    X(8, 288, 4, 6, 12, 24)          \
    X(8, 324, 6, 6, 9, 18)           \
    X(9, 384, 8, 8, 6, 16)           \
    X(10, 432, 12, 6, 6, 36)         \
    X(10, 486, 6, 9, 9, 27)

// Alternative plans with fewer elements per thread (for register-heavy
// passes), chosen per pass by the tuner.
#define CBS_PLANS_WIDE(X)            \
    X(1, 64, 4, 4, 4, 16)            \
    X(2, 128, 4, 4, 8, 16)           \
    X(3, 256, 4, 8, 8, 32)

#define CBS_PLAN_GROUPS 11

// Groups below this one compile every pass variant the tuner chooses from
// (LDS layouts of the propagator pass, prefetch of the last-axis inverse
// pass); the lengths of the later groups, off the benchmarked shapes, compile
// the baseline variant of each pass only.
#define CBS_FULL_VARIANT_GROUPS 5
