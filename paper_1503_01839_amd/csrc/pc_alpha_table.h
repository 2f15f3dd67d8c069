// pc_alpha_table.h -- alpha = y / icbrt(x) and the sieve shape per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {
    double log10x;
    double alpha;
    unsigned seg_kib; // LDS segment, KiB
    unsigned wg;      // workgroup threads
};

static const pc_alpha_entry kAlphaTable[] = {
    {7.0, 48, 32, 512}, // 0.33 ms
    {7.5, 32, 32, 512}, // 0.35 ms
    {8.0, 48, 32, 512}, // 0.37 ms
    {8.5, 32, 32, 512}, // 0.40 ms
    {9.0, 16, 64, 1024}, // 0.45 ms
    {9.5, 12, 64, 1024}, // 0.54 ms
    {10.0, 8, 64, 1024}, // 0.71 ms
    {10.5, 8, 64, 1024}, // 0.92 ms
    {11.0, 12, 64, 1024}, // 1.23 ms
    {11.5, 6, 32, 512}, // 1.76 ms
    {12.0, 8, 32, 512}, // 2.39 ms
    {12.5, 8, 32, 512}, // 2.32 ms
    {13.0, 6, 32, 512}, // 2.77 ms
    {13.5, 6, 32, 512}, // 3.17 ms
    {14.0, 3, 32, 512}, // 3.41 ms
    {14.5, 2, 32, 512}, // 3.87 ms
    {15.0, 4, 32, 512}, // 5.11 ms
    {15.5, 4, 32, 512}, // 6.58 ms
    {16.0, 8, 32, 512}, // 8.39 ms
    {16.5, 12, 32, 512}, // 11.75 ms
    {17.0, 24, 32, 512}, // 23.16 ms
    {17.5, 24, 32, 512}, // 44.86 ms
    {18.0, 24, 32, 512}, // 98.07 ms
    {18.5, 32, 32, 512}, // 204.87 ms
    {19.0, 32, 32, 512}, // 431.06 ms
};
