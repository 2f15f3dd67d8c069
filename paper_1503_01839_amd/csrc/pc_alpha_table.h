// pc_alpha_table.h -- alpha = y / icbrt(x) per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {
    double log10x;
    double alpha;
};

static const pc_alpha_entry kAlphaTable[] = {
    {7.0, 24}, // 0.33 ms
    {7.5, 16}, // 0.37 ms
    {8.0, 8}, // 0.42 ms
    {8.5, 6}, // 0.51 ms
    {9.0, 3}, // 0.62 ms
    {9.5, 2}, // 0.78 ms
    {10.0, 1.5}, // 1.00 ms
    {10.5, 1.5}, // 1.29 ms
    {11.0, 2}, // 1.75 ms
    {11.5, 1.5}, // 2.33 ms
    {12.0, 4}, // 2.63 ms
    {12.5, 4}, // 3.40 ms
    {13.0, 3}, // 3.33 ms
    {13.5, 2}, // 3.69 ms
    {14.0, 3}, // 3.98 ms
    {14.5, 2}, // 4.27 ms
    {15.0, 4}, // 7.98 ms
    {15.5, 6}, // 9.79 ms
    {16.0, 8}, // 13.24 ms
    {16.5, 12}, // 27.78 ms
    {17.0, 12}, // 58.88 ms
    {17.5, 16}, // 125.78 ms
    {18.0, 16}, // 264.63 ms
    {18.5, 16}, // 585.45 ms
    {19.0, 24}, // 1258.44 ms
};
