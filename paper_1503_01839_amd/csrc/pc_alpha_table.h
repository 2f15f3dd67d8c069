// pc_alpha_table.h -- alpha = y / icbrt(x) and the sieve shape per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {
    double log10x;
    double alpha;       // least time for one query
    unsigned seg_kib;   // LDS segment, KiB
    unsigned wg;        // workgroup threads
    double batch_alpha; // least time for a batch of queries of this size
};

static const pc_alpha_entry kAlphaTable[] = {
    {7.0, 1, 32, 512, 1}, // 0.41 ms
    {7.5, 24, 32, 512, 4}, // 0.44 ms
    {8.0, 32, 32, 512, 1}, // 0.47 ms
    {8.5, 16, 32, 512, 4}, // 0.51 ms
    {9.0, 24, 64, 1024, 3}, // 0.57 ms
    {9.5, 24, 32, 512, 8}, // 0.63 ms
    {10.0, 48, 64, 1024, 12}, // 0.68 ms
    {10.5, 48, 64, 1024, 8}, // 0.73 ms
    {11.0, 48, 64, 1024, 8}, // 0.79 ms
    {11.5, 16, 32, 512, 3}, // 0.89 ms
    {12.0, 6, 32, 512, 6}, // 0.94 ms
    {12.5, 4, 32, 512, 8}, // 0.97 ms
    {13.0, 2, 32, 512, 8}, // 1.12 ms
    {13.5, 4, 32, 512, 8}, // 1.26 ms
    {14.0, 6, 32, 512, 12}, // 1.52 ms
    {14.5, 12, 32, 512, 16}, // 2.00 ms
    {15.0, 12, 32, 512, 16}, // 2.80 ms
    {15.5, 12, 32, 512, 16}, // 4.07 ms
    {16.0, 16, 32, 512, 24}, // 6.28 ms
    {16.5, 16, 32, 512, 16}, // 9.83 ms
    {17.0, 24, 32, 512, 24}, // 19.10 ms
    {17.5, 24, 32, 512, 24}, // 35.96 ms
    {18.0, 24, 32, 512, 24}, // 78.00 ms
    {18.5, 32, 32, 512, 32}, // 157.40 ms
    {19.0, 32, 32, 512, 32}, // 325.65 ms
};
