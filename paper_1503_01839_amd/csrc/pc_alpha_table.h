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
    {7.0, 32, 32, 512, 1}, // 0.39 ms
    {7.5, 32, 32, 512, 8}, // 0.40 ms
    {8.0, 12, 32, 512, 1}, // 0.43 ms
    {8.5, 48, 32, 512, 1.5}, // 0.47 ms
    {9.0, 16, 64, 1024, 3}, // 0.52 ms
    {9.5, 48, 64, 1024, 8}, // 0.57 ms
    {10.0, 24, 64, 1024, 6}, // 0.62 ms
    {10.5, 8, 32, 512, 8}, // 0.66 ms
    {11.0, 16, 32, 512, 8}, // 0.72 ms
    {11.5, 1.5, 32, 512, 6}, // 0.76 ms
    {12.0, 2, 32, 512, 12}, // 0.80 ms
    {12.5, 4, 32, 512, 8}, // 0.85 ms
    {13.0, 2, 32, 512, 8}, // 0.97 ms
    {13.5, 2, 32, 512, 12}, // 1.12 ms
    {14.0, 6, 32, 512, 12}, // 1.36 ms
    {14.5, 8, 32, 512, 12}, // 1.71 ms
    {15.0, 12, 32, 512, 16}, // 2.29 ms
    {15.5, 12, 32, 512, 16}, // 3.33 ms
    {16.0, 16, 32, 512, 24}, // 5.29 ms
    {16.5, 16, 32, 512, 16}, // 8.75 ms
    {17.0, 24, 32, 512, 24}, // 17.06 ms
    {17.5, 24, 32, 512, 24}, // 33.92 ms
    {18.0, 28, 32, 512, 28}, // 69.34 ms
    {18.5, 32, 32, 512, 32}, // 144.61 ms
    {19.0, 32, 32, 512, 32}, // 308.42 ms
};
