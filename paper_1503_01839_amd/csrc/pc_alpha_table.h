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
    {7.0, 16, 32, 512, 1}, // 0.38 ms
    {7.5, 32, 32, 512, 4}, // 0.40 ms
    {8.0, 12, 32, 512, 1}, // 0.43 ms
    {8.5, 8, 32, 512, 2}, // 0.48 ms
    {9.0, 8, 32, 512, 3}, // 0.53 ms
    {9.5, 32, 32, 512, 8}, // 0.60 ms
    {10.0, 36, 64, 1024, 12}, // 0.62 ms
    {10.5, 8, 32, 512, 8}, // 0.67 ms
    {11.0, 16, 32, 512, 8}, // 0.73 ms
    {11.5, 1.5, 32, 512, 6}, // 0.77 ms
    {12.0, 2, 32, 512, 12}, // 0.82 ms
    {12.5, 4, 32, 512, 8}, // 0.86 ms
    {13.0, 6, 32, 512, 8}, // 1.01 ms
    {13.5, 4, 32, 512, 12}, // 1.14 ms
    {14.0, 6, 32, 512, 16}, // 1.38 ms
    {14.5, 8, 32, 512, 16}, // 1.73 ms
    {15.0, 12, 32, 512, 24}, // 2.33 ms
    {15.5, 12, 32, 512, 24}, // 3.37 ms
    {16.0, 16, 32, 512, 24}, // 5.27 ms
    {16.5, 16, 32, 512, 16}, // 8.72 ms
    {17.0, 24, 32, 512, 24}, // 16.05 ms
    {17.5, 32, 32, 512, 32}, // 31.61 ms
    {18.0, 36, 32, 512, 36}, // 64.94 ms
    {18.5, 40, 32, 512, 40}, // 134.61 ms
    {19.0, 48, 32, 512, 48}, // 281.39 ms
};
